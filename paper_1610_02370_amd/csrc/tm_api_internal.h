// Host-side state shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <mutex>
#include <vector>

#include "../../include/tm.h"
#include "tm_internal.h"

namespace tmsap {

// Grow-only device allocation.
struct DeviceBuffer {
    void* ptr = nullptr;
    size_t bytes = 0;
    ~DeviceBuffer();
    hipError_t ensure(size_t n);
    void release();
};

struct GaugeEntry {
    const void* U = nullptr;
    unsigned long long tag = 0;
    double kappa = 0, csw = 0;
    Geo g{};
    GaugeDev dev;
    EoCache eo;                        // even-odd site inverses derived from dev.clover
    unsigned long long last_call = 0;  // call that last used this entry (never evicted by that call)
    ~GaugeEntry();
};

struct DeviceState {
    int device = 0;
    unsigned long long call_id = 0;  // bumped by every entry point
    std::mutex mutex;
    std::vector<std::unique_ptr<GaugeEntry>> gauge;
    DeviceBuffer stats;   // small flags / reductions
    DeviceBuffer io;      // canonical <-> internal staging
    DeviceBuffer solver;  // Krylov bases and solver vectors
    DeviceBuffer red;     // reduction partials
};

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* where);
// Per-device state of the current device; every entry point gets it through
// this call, which also starts a new call id for the gauge cache.
DeviceState* device_state(int* err);
int check_geom(const tm_geom* geom);
int check_opts(const tm_opts* opts);
int choose_tile(const tm_geom* geom, const int* req, int tile[4]);
int check_sap_blocks(const tm_geom* geom, const int* block_dims, int tile[4]);
Geo make_geo(const tm_geom* geom, const int tile[4]);
Prec clover_prec_for(Prec link_p);
int get_gauge(DeviceState* ds, const Geo& g, const void* U, double kappa, double csw, Prec link_p,
              unsigned long long tag, hipStream_t st, const GaugeDev** out);
// Gauge cache entries: whether G is still held, and dropping it (frees its memory).
bool gauge_held(DeviceState* ds, const GaugeDev* G);
void drop_gauge(DeviceState* ds, const GaugeDev* G);
// SAP tuning cache: the stored (block shape, systems per workgroup) for this
// problem, if any; returns false when nothing is stored.
bool tune_lookup(const tm_geom* geom, int storage, int n_cycles, int mr_iters, int eo, int block[4], int* sys_tile);
SpinorBuf wrap_internal(void* base, const Geo& g, int nsys, Prec p);
size_t internal_bytes(const Geo& g, int nsys, Prec p);
void fill_mu(const tm_geom* geom, double* mu);
// Site-diagonal inverse sets (A + i mu Gamma5)^-1 at the sites of one parity for
// the systems' |mu| values, cached with G; sel[k] picks system k's set, bit k of
// *adj marks mu_k < 0 (use the adjoint).
int prepare_site_inverses(const Geo& g, const GaugeDev& G, const double* mu, int nsys, int parity, hipStream_t st,
                          const void* inv[kMaxEoMu], unsigned char sel[kMaxSys], unsigned long long* adj);
// Largest group of systems (at most `group` when positive) whose per-system
// workspace fits in 92 % of the free device memory plus the solver buffer and
// `reusable` bytes the caller already holds for the same purpose.
int fit_group(DeviceState* ds, int nsys, int group, size_t per_sys, size_t fixed, size_t reusable = 0);
// n_cycles red-black SAP cycles; eo selects even-odd preconditioned block
// solves (site inverses built on first use for each |mu| and kept with G).
// With w_out (only where sap_fills_w holds), the last half-sweep also writes
// D x on its blocks (colour 1) to w_out; run_dirac_colour(..., 0) completes it.
int run_sap(const Geo& g, const GaugeDev& G, const SpinorBuf& b, const SpinorBuf& x, const double* mu, int nsys,
            int n_cycles, int mr_iters, bool x_zero, int sys_tile, hipStream_t st, bool eo = false,
            void* w_out = nullptr);
int run_dirac(const Geo& g, const GaugeDev& G, const SpinorBuf& in, const SpinorBuf& out, const double* mu, int nsys,
              Prec compute, hipStream_t st);
// out = D in on the 4^4 blocks of one colour only (FP32 tiled operator; other blocks untouched).
int run_dirac_colour(const Geo& g, const GaugeDev& G, const SpinorBuf& in, const SpinorBuf& out, const double* mu,
                     int nsys, int colour, hipStream_t st);

// Device address of the current device's fixed scratch array of the no-allocation entry point
// (tm_noalloc.hip), looked up once per device; out may be NULL (set-up only).
int noalloc_scratch(void** out);

// ---- two-level method (tm_mg_api.cpp)
// z = the handle's two-level preconditioner applied to r: FP32 internal fields
// of ns systems tiled by the handle's aggregates (the handle holds its gauge copy).
int mg_apply(tm_mg* mg, DeviceState* ds, const SpinorBuf& r, const SpinorBuf& z, const double* mu, int ns,
             hipStream_t st);
// TM_OK when geom has the handle's dims, boundary phases and shifts and its device is current.
int mg_matches(const tm_mg* mg, const tm_geom* geom);
void mg_block_dims(const tm_mg* mg, int bd[4]);
// device bytes per system of one preconditioner application (coarse vectors and Krylov basis)
size_t mg_workspace_per_sys(const tm_mg* mg);
// device bytes of that workspace the handle holds now
size_t mg_workspace_held(const tm_mg* mg);

}  // namespace tmsap
