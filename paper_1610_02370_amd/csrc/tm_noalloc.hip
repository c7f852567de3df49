// SAP smoothing without device allocation: tm_sap_smooth_noalloc.
//
// Everything the smoother needs beyond the caller's buffers (the link copy,
// the clover term, the internal copies of b and x, the validation flags)
// lives in one file-scope device array, `scratch`, of kScratchBytes per GPU.
// Host code never passes the array's name to a kernel: each device's copy of
// the array has its own address, fetched once per device with
// hipGetSymbolAddress and kept in g_scratch.  Every call on a device reuses
// that device's array and leaves the last call's contents in it, so calls
// that overlap on one device race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/tm.h"
#include "tm_api_internal.h"

namespace tmsap {

constexpr size_t kScratchBytes = (size_t)TM_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch is carved in 256-byte units");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch[kMaxDevices] = {};

// Clears n words (the validation flags) with a kernel rather than a memset node.
__global__ void k_clear_words(unsigned* p, int n) {
    const int i = threadIdx.x;
    if (i < n) p[i] = 0u;
}

}  // namespace

// Device address of the current device's scratch array, looked up on first use.
int noalloc_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(TM_ERR_ARG, "device %d beyond the library's %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(TM_ERR_HIP, "hipGetSymbolAddress(scratch) returned a null address");
        g_scratch[dev] = p;
    }
    if (out) *out = g_scratch[dev];
    return TM_OK;
}

}  // namespace tmsap

using namespace tmsap;

extern "C" {

int tm_sap_smooth_noalloc(const tm_geom* geom, const void* U, const void* b, void* x, double kappa, double c_sw,
                          const int block_dims[4], int n_cycles, int mr_iters, const tm_opts* opts) {
    int rc;
    if ((rc = check_geom(geom)) || (rc = check_opts(opts))) return rc;
    if (!U || !b || !x) return fail(TM_ERR_ARG, "null pointer");
    if (b == x) return fail(TM_ERR_ARG, "b and x alias");
    if (n_cycles < 0 || mr_iters < 0) return fail(TM_ERR_ARG, "negative cycle or MR count");
    if (!(kappa > 0) || !std::isfinite(kappa) || !std::isfinite(c_sw)) return fail(TM_ERR_ARG, "bad kappa or c_sw");
    if (opts->sap_eo) return fail(TM_ERR_ARG, "the no-allocation smoother has no even-odd block solves");
    int tile[4];
    if ((rc = check_sap_blocks(geom, block_dims, tile))) return rc;
    const Prec sp = (Prec)opts->storage, cp = clover_prec_for(sp);
    if (!sap_supported(sp, sp, cp, (Prec)opts->compute))
        return fail(TM_ERR_PREC, "unsupported precision combination for SAP");
    const Geo g = make_geo(geom, tile);
    const bool canonical = opts->io == TM_IO_CANONICAL;

    // scratch carving: flags | links | clover | b | x (internal copies only for canonical buffers)
    const size_t flags_b = 256;
    const size_t links_b = align256((size_t)4 * 3 * g.V * unit_bytes(sp));
    const size_t clover_b = align256((size_t)18 * g.V * unit_bytes(cp));
    const size_t spinor_b = canonical ? internal_bytes(g, geom->nsys, sp) : 0;
    const size_t need = flags_b + links_b + clover_b + 2 * spinor_b;
    if (need > kScratchBytes)
        return fail(TM_ERR_ARG,
                    "this call needs %zu bytes of scratch (links, clover%s); tm_sap_smooth_noalloc holds %zu "
                    "(use tm_sap_smooth)",
                    need, canonical ? ", internal b and x" : "", kScratchBytes);
    void* base = nullptr;
    if ((rc = noalloc_scratch(&base))) return rc;
    char* p = static_cast<char*>(base);
    unsigned* flags = reinterpret_cast<unsigned*>(p);
    p += flags_b;
    GaugeDev G;
    G.links = p;
    p += links_b;
    G.clover = p;
    p += clover_b;
    G.link_prec = sp;
    G.clover_prec = cp;
    G.eo = nullptr;

    hipStream_t st = (hipStream_t)opts->stream;
    hipError_t h;
    // the gauge copy and clover term, validated as tm_sap_smooth validates them
    hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, st, flags, 4);
    if ((h = hipGetLastError()) != hipSuccess) return hip_fail(h, "clear flags");
    if ((h = launch_link_ingest(g, sp, U, G.links, flags, st)) != hipSuccess) return hip_fail(h, "link ingest");
    if ((h = launch_clover_build(g, cp, U, 1.0 / (2.0 * kappa), c_sw, G.clover, st)) != hipSuccess)
        return hip_fail(h, "clover build");
    unsigned host[2];
    if ((h = hipMemcpyAsync(host, flags, sizeof host, hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(h, "flags copy");
    if ((h = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(h, "gauge ingest");
    if (host[1]) return fail(TM_ERR_NONFINITE, "gauge field holds NaN or Inf");
    float dev;
    std::memcpy(&dev, &host[0], sizeof dev);
    if (!(dev <= 1e-6f)) return fail(TM_ERR_NOT_SU3, "links deviate from SU(3) by %g (limit 1e-6)", (double)dev);

    double mu[kMaxSys];
    fill_mu(geom, mu);
    if (!canonical) {
        SpinorBuf bb = wrap_internal(const_cast<void*>(b), g, geom->nsys, sp);
        SpinorBuf xx = wrap_internal(x, g, geom->nsys, sp);
        return run_sap(g, G, bb, xx, mu, geom->nsys, n_cycles, mr_iters, false, opts->sys_tile, st, false);
    }
    SpinorBuf bb = wrap_internal(p, g, geom->nsys, sp);
    SpinorBuf xx = wrap_internal(p + spinor_b, g, geom->nsys, sp);
    if ((h = launch_spinor_import(g, bb, b, flags + 2, st)) != hipSuccess) return hip_fail(h, "spinor import");
    if ((h = launch_spinor_import(g, xx, x, flags + 2, st)) != hipSuccess) return hip_fail(h, "spinor import");
    if ((rc = run_sap(g, G, bb, xx, mu, geom->nsys, n_cycles, mr_iters, false, opts->sys_tile, st, false)))
        return rc;
    if ((h = launch_spinor_export(g, xx, x, st)) != hipSuccess) return hip_fail(h, "spinor export");
    return TM_OK;
}

}  // extern "C"
