// SAP tuner: picks the Schwarz block shape and the number of systems per
// workgroup that give the highest smoother throughput for one problem size,
// and keeps the choice in a small text cache.
//
// The paper fixes 4^4 blocks (Table 1) for its machine; on another chip the
// best shape depends on the on-chip memory per workgroup and on how many
// blocks fill the device, so it is measured.  Only throughput is measured:
// the block shape also changes the preconditioner (section 2.4), so a solve
// with a tuned shape can take a different number of iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tm.h"
#include "tm_api_internal.h"
#include "tm_blas.h"

namespace tmsap {

namespace {

std::mutex g_tune_mutex;

std::string cache_path() {
    const char* p = std::getenv("TM_TUNE_CACHE");
    return (p && *p) ? std::string(p) : std::string("tm_tune.txt");
}

// One cache line: key fields then the choice.
//   sap T Z Y X nsys storage cycles mr antiperiodic_t eo : b0 b1 b2 b3 tile seconds
std::string cache_key(const tm_geom* geom, int storage, int n_cycles, int mr_iters, int eo) {
    char k[160];
    std::snprintf(k, sizeof k, "sap %d %d %d %d %d %d %d %d %d %d", geom->dims[0], geom->dims[1], geom->dims[2],
                  geom->dims[3], geom->nsys, storage, n_cycles, mr_iters, geom->antiperiodic_t ? 1 : 0, eo);
    return k;
}

bool valid_shape(const tm_geom* geom, const int b[4]) {
    long long vb = 1;
    for (int a = 0; a < 4; ++a) {
        if (b[a] <= 0 || geom->dims[a] % b[a] != 0 || (geom->dims[a] / b[a]) % 2 != 0) return false;
        vb *= b[a];
    }
    return vb <= 256;
}

// Candidate shapes: extents from {2,3,4,6,8} with 64..256 sites and an aspect
// ratio of at most 4; on lattices too small for any of those, every valid
// shape of 16..256 sites with extents up to 8.
std::vector<std::array<int, 4>> candidates(const tm_geom* geom, bool eo) {
    std::vector<std::array<int, 4>> out;
    const int ext[] = {2, 3, 4, 6, 8};
    for (int pass = 0; pass < 2 && out.empty(); ++pass) {
        const int lo = pass == 0 ? 64 : 16;
        for (int i0 = 0; i0 < 8; ++i0)
            for (int i1 = 0; i1 < 8; ++i1)
                for (int i2 = 0; i2 < 8; ++i2)
                    for (int i3 = 0; i3 < 8; ++i3) {
                        int b[4];
                        const int idx[4] = {i0, i1, i2, i3};
                        bool ok = true;
                        for (int a = 0; a < 4; ++a) {
                            if (pass == 0) {
                                if (idx[a] >= 5) ok = false;
                                else b[a] = ext[idx[a]];
                            } else {
                                b[a] = idx[a] + 1;
                            }
                        }
                        if (!ok || !valid_shape(geom, b)) continue;
                        if (eo && b[3] % 2 != 0) continue;  // even-odd pairs sites along x
                        const int vb = b[0] * b[1] * b[2] * b[3];
                        const int mx = std::max(std::max(b[0], b[1]), std::max(b[2], b[3]));
                        const int mn = std::min(std::min(b[0], b[1]), std::min(b[2], b[3]));
                        if (vb < lo) continue;
                        if (pass == 0 && mx > 4 * mn) continue;
                        out.push_back({b[0], b[1], b[2], b[3]});
                    }
    }
    return out;
}

struct Timing {
    int rc = TM_OK;
    double seconds = 0;  // per SAP application
};

// Time SAP applications of one configuration (zero initial guess, as the
// preconditioner applies it).  b and x live in the device's staging buffer.
Timing time_config(DeviceState* ds, const tm_geom* geom, const void* U, double kappa, double c_sw, int n_cycles,
                   int mr_iters, Prec sp, bool eo, unsigned long long tag, hipStream_t st, const int block[4],
                   int sys_tile) {
    Timing t;
    Geo g = make_geo(geom, block);
    const GaugeDev* G = nullptr;
    std::vector<const GaugeDev*> before;
    {
        std::lock_guard<std::mutex> lock(ds->mutex);
        for (auto& e : ds->gauge) before.push_back(&e->dev);
    }
    if ((t.rc = get_gauge(ds, g, U, kappa, c_sw, sp, tag, st, &G))) return t;
    const bool fresh = std::find(before.begin(), before.end(), G) == before.end();
    struct Drop {
        DeviceState* ds;
        const GaugeDev* G;
        bool on;
        ~Drop() {
            if (on && gauge_held(ds, G)) drop_gauge(ds, G);
        }
    } drop{ds, G, fresh};

    const size_t nb = internal_bytes(g, geom->nsys, sp);
    hipError_t h = ds->io.ensure(2 * nb);
    if (h != hipSuccess) {
        t.rc = hip_fail(h, "tuning workspace");
        return t;
    }
    SpinorBuf bb = wrap_internal(ds->io.ptr, g, geom->nsys, sp);
    SpinorBuf xx = wrap_internal(static_cast<char*>(ds->io.ptr) + nb, g, geom->nsys, sp);
    if ((h = blas_fill_pattern(bb, g.V, 0x5A17u, st)) != hipSuccess ||
        (h = blas_fill_pattern(xx, g.V, 0x0u, st)) != hipSuccess) {
        t.rc = hip_fail(h, "tuning inputs");
        return t;
    }
    double mu[kMaxSys];
    fill_mu(geom, mu);
    hipEvent_t e0, e1;
    if ((h = hipEventCreate(&e0)) != hipSuccess) {
        t.rc = hip_fail(h, "event");
        return t;
    }
    if ((h = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        t.rc = hip_fail(h, "event");
        return t;
    }
    auto run = [&](int reps, double* sec) -> int {
        int rc;
        hipError_t hh;
        if ((hh = hipEventRecord(e0, st)) != hipSuccess) return hip_fail(hh, "event");
        for (int r = 0; r < reps; ++r)
            if ((rc = run_sap(g, *G, bb, xx, mu, geom->nsys, n_cycles, mr_iters, true, sys_tile, st, eo))) return rc;
        if ((hh = hipEventRecord(e1, st)) != hipSuccess) return hip_fail(hh, "event");
        if ((hh = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(hh, "SAP timing");
        float ms = 0;
        if ((hh = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return hip_fail(hh, "event");
        *sec = ms * 1e-3 / reps;
        return TM_OK;
    };
    double first = 0;
    if ((t.rc = run(1, &first)) == TM_OK) {
        // about 50 ms of timed work per configuration, at least 2 and at most 10 applications
        const int reps = std::max(2, std::min(10, (int)std::ceil(0.05 / std::max(first, 1e-6))));
        t.rc = run(reps, &t.seconds);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return t;
}

}  // namespace

bool tune_lookup(const tm_geom* geom, int storage, int n_cycles, int mr_iters, int eo, int block[4], int* sys_tile) {
    // solves consult a cache only when the caller names one: the same call then gives the
    // same block shape (and preconditioner) whatever the working directory holds
    const char* named = std::getenv("TM_TUNE_CACHE");
    if (!named || !*named) return false;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    FILE* f = std::fopen(cache_path().c_str(), "r");
    if (!f) return false;
    const std::string key = cache_key(geom, storage, n_cycles, mr_iters, eo) + " :";
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, key.c_str(), key.size()) != 0) continue;
        int b[4], tile;
        if (std::sscanf(line + key.size(), "%d %d %d %d %d", &b[0], &b[1], &b[2], &b[3], &tile) != 5) continue;
        if (!valid_shape(geom, b) || tile < 0 || (eo && b[3] % 2 != 0)) continue;
        std::memcpy(block, b, sizeof b);
        *sys_tile = tile;
        found = true;  // the last valid line wins
    }
    std::fclose(f);
    return found;
}

}  // namespace tmsap

using namespace tmsap;

extern "C" {

int tm_autotune_sap(const tm_geom* geom, const void* U, double kappa, double c_sw, int n_cycles, int mr_iters,
                    const tm_opts* opts, int best_block[4], int* best_sys_tile) {
    int rc;
    if ((rc = check_geom(geom)) || (rc = check_opts(opts))) return rc;
    if (!U || !best_block || !best_sys_tile) return fail(TM_ERR_ARG, "null pointer");
    if (n_cycles < 1 || mr_iters < 0) return fail(TM_ERR_ARG, "bad cycle or MR count");
    if (!(kappa > 0) || !std::isfinite(kappa) || !std::isfinite(c_sw)) return fail(TM_ERR_ARG, "bad kappa or c_sw");
    const Prec sp = (Prec)opts->storage;
    const bool eo = opts->sap_eo != 0;
    if (!sap_supported(sp, sp, clover_prec_for(sp), sp == P_F64 ? P_F64 : P_F32))
        return fail(TM_ERR_PREC, "unsupported precision combination for SAP");
    std::vector<std::array<int, 4>> cand = candidates(geom, eo);
    if (cand.empty()) return fail(TM_ERR_BLOCKS, "no block shape of 16..256 sites fits these dims");
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    hipStream_t st = (hipStream_t)opts->stream;

    // stage 1: block shape with all systems in one workgroup; stage 2: systems per workgroup for that shape
    double best = 0;
    int bb[4] = {0, 0, 0, 0}, btile = 0;
    for (auto& c : cand) {
        Timing t = time_config(ds, geom, U, kappa, c_sw, n_cycles, mr_iters, sp, eo, opts->gauge_tag, st, c.data(), 0);
        if (t.rc == TM_ERR_BLOCKS) continue;  // shape needs more on-chip memory than the device has
        if (t.rc) return t.rc;
        if (bb[0] == 0 || t.seconds < best) {
            best = t.seconds;
            std::memcpy(bb, c.data(), sizeof bb);
        }
    }
    if (bb[0] == 0) return fail(TM_ERR_BLOCKS, "no candidate block shape could be launched");
    std::vector<int> tried{geom->nsys};
    for (int split : {2, 3, 4, 6}) {
        const int tile = (geom->nsys + split - 1) / split;
        if (std::find(tried.begin(), tried.end(), tile) != tried.end()) continue;
        tried.push_back(tile);
        Timing t = time_config(ds, geom, U, kappa, c_sw, n_cycles, mr_iters, sp, eo, opts->gauge_tag, st, bb, tile);
        if (t.rc) return t.rc;
        if (t.seconds < best) {
            best = t.seconds;
            btile = tile;
        }
    }
    std::memcpy(best_block, bb, sizeof bb);
    *best_sys_tile = btile;

    std::lock_guard<std::mutex> lock(g_tune_mutex);
    FILE* f = std::fopen(cache_path().c_str(), "a");
    if (f) {
        std::fprintf(f, "%s : %d %d %d %d %d %.6e\n", cache_key(geom, (int)sp, n_cycles, mr_iters, eo ? 1 : 0).c_str(), bb[0],
                     bb[1], bb[2], bb[3], btile, best);
        std::fclose(f);
    }
    return TM_OK;
}

}  // extern "C"
