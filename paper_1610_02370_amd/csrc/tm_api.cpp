// C ABI of the library: argument checking, the per-device gauge cache,
// workspaces, and the entry points declared in include/tm.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tm.h"
#include "tm_api_internal.h"

namespace tmsap {

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* where) {
    if (e == hipErrorOutOfMemory) return fail(TM_ERR_NOMEM, "%s: out of device memory", where);
    return fail(TM_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

// ------------------------------------------------------------------ state

static std::mutex g_mutex;
static std::vector<std::unique_ptr<DeviceState>> g_devices;

DeviceState* device_state(int* err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *err = hip_fail(e, "hipGetDevice");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    for (auto& d : g_devices)
        if (d->device == dev) {
            ++d->call_id;
            return d.get();
        }
    g_devices.emplace_back(new DeviceState());
    g_devices.back()->device = dev;
    g_devices.back()->call_id = 1;
    return g_devices.back().get();
}

DeviceBuffer::~DeviceBuffer() { release(); }
void DeviceBuffer::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}
hipError_t DeviceBuffer::ensure(size_t n) {
    if (n <= bytes) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&ptr, n);
    if (e != hipSuccess) {
        ptr = nullptr;
        return e;
    }
    bytes = n;
    return hipSuccess;
}

void EoCache::release() {
    for (int k = 0; k < n; ++k)
        if (inv[k]) (void)hipFree(inv[k]);
    n = 0;
}

GaugeEntry::~GaugeEntry() {
    if (dev.links) (void)hipFree(dev.links);
    if (dev.clover) (void)hipFree(dev.clover);
}

// ------------------------------------------------------------------ checks

static bool prec_ok(int p) { return p >= TM_F64 && p <= TM_BF16; }

int check_geom(const tm_geom* geom) {
    if (!geom) return fail(TM_ERR_ARG, "geom is NULL");
    for (int a = 0; a < 4; ++a)
        if (geom->dims[a] <= 0) return fail(TM_ERR_DIMS, "dims[%d] = %d is not positive", a, geom->dims[a]);
    long long V = (long long)geom->dims[0] * geom->dims[1] * geom->dims[2] * geom->dims[3];
    if (V > (1LL << 31) / 4) return fail(TM_ERR_DIMS, "lattice of %lld sites is too large", V);
    if (geom->nsys < 1 || geom->nsys > TM_MAX_SYS)
        return fail(TM_ERR_ARG, "nsys = %d outside 1..%d", geom->nsys, TM_MAX_SYS);
    if (!geom->mu) return fail(TM_ERR_ARG, "geom->mu is NULL");
    for (int a = 0; a < 4; ++a)
        if (!std::isfinite(geom->theta[a])) return fail(TM_ERR_NONFINITE, "theta[%d] is not finite", a);
    if (!std::isfinite(geom->mu_shift[0]) || !std::isfinite(geom->mu_shift[1]))
        return fail(TM_ERR_NONFINITE, "mu_shift is not finite");
    for (int k = 0; k < geom->nsys; ++k)
        if (!std::isfinite(geom->mu[k])) return fail(TM_ERR_NONFINITE, "mu[%d] is not finite", k);
    return TM_OK;
}

int check_opts(const tm_opts* opts) {
    if (!opts) return fail(TM_ERR_ARG, "opts is NULL");
    if (!prec_ok(opts->storage) || !prec_ok(opts->compute)) return fail(TM_ERR_PREC, "unknown precision");
    if (opts->compute != TM_F64 && opts->compute != TM_F32) return fail(TM_ERR_PREC, "compute must be F64 or F32");
    if (opts->storage == TM_F64 && opts->compute != TM_F64)
        return fail(TM_ERR_PREC, "FP64 storage requires FP64 compute");
    if (opts->storage != TM_F64 && opts->compute != TM_F32)
        return fail(TM_ERR_PREC, "FP32/FP16/BF16 storage computes in FP32");
    if (opts->io != TM_IO_CANONICAL && opts->io != TM_IO_INTERNAL) return fail(TM_ERR_ARG, "unknown io mode");
    if (opts->sys_tile < 0) return fail(TM_ERR_ARG, "sys_tile must be >= 0");
    if (opts->sap_eo != 0 && opts->sap_eo != 1) return fail(TM_ERR_ARG, "sap_eo must be 0 or 1");
    return TM_OK;
}

// Tile for a layout: explicit, else 4 where it divides the axis, else 2, else 1.
int choose_tile(const tm_geom* geom, const int* req, int tile[4]) {
    bool given = req && (req[0] | req[1] | req[2] | req[3]);
    for (int a = 0; a < 4; ++a) {
        if (given) {
            tile[a] = req[a];
            if (tile[a] <= 0 || geom->dims[a] % tile[a] != 0)
                return fail(TM_ERR_DIMS, "block/tile %d does not divide dims[%d] = %d", tile[a], a, geom->dims[a]);
        } else {
            tile[a] = geom->dims[a] % 4 == 0 ? 4 : (geom->dims[a] % 2 == 0 ? 2 : 1);
        }
    }
    if ((long long)tile[0] * tile[1] * tile[2] * tile[3] > 1024) return fail(TM_ERR_BLOCKS, "tile holds more than 1024 sites");
    return TM_OK;
}

Geo make_geo(const tm_geom* geom, const int tile[4]) {
    Geo g;
    g.V = 1;
    g.Vb = 1;
    for (int a = 0; a < 4; ++a) {
        g.d[a] = geom->dims[a];
        g.lb[a] = tile[a];
        g.nb[a] = geom->dims[a] / tile[a];
        g.V *= geom->dims[a];
        g.Vb *= tile[a];
    }
    for (int mu = 0; mu < 4; ++mu) {
        double th = geom->theta[mu];
        if (mu == 0 && geom->antiperiodic_t) th += M_PI;
        g.bcr[mu] = std::cos(th);
        g.bci[mu] = std::sin(th);
        if (geom->theta[mu] == 0.0) {  // exact signs for the plain boundaries
            g.bcr[mu] = (mu == 0 && geom->antiperiodic_t) ? -1.0 : 1.0;
            g.bci[mu] = 0.0;
        }
        g.bcrf[mu] = (float)g.bcr[mu];
        g.bcif[mu] = (float)g.bci[mu];
    }
    g.mu_shift[0] = geom->mu_shift[0];
    g.mu_shift[1] = geom->mu_shift[1];
    return g;
}

Prec clover_prec_for(Prec link_p) { return (link_p == P_F16 || link_p == P_BF16) ? P_F32 : link_p; }

// Links + clover derived from U at (link precision, tile).  A nonzero tag
// reuses a copy made for the same (U, tag, dims, tile, kappa, c_sw,
// precision); tag 0 rebuilds into a reusable tag-0 slot of matching size.
static bool same_shape(const GaugeEntry& e, const Geo& g, Prec link_p) {
    return e.dev.link_prec == link_p && std::memcmp(e.g.d, g.d, sizeof g.d) == 0 &&
           std::memcmp(e.g.lb, g.lb, sizeof g.lb) == 0;
}

int get_gauge(DeviceState* ds, const Geo& g, const void* U, double kappa, double csw, Prec link_p,
              unsigned long long tag, hipStream_t st, const GaugeDev** out) {
    const Prec cl_p = clover_prec_for(link_p);
    std::lock_guard<std::mutex> lock(ds->mutex);
    GaugeEntry* slot = nullptr;
    for (auto& ep : ds->gauge) {
        GaugeEntry& e = *ep;
        if (!same_shape(e, g, link_p)) continue;
        if (tag != 0 && e.tag == tag && e.U == U && e.kappa == kappa && e.csw == csw) {
            e.last_call = ds->call_id;
            *out = &e.dev;
            return TM_OK;
        }
        if (tag == 0 && e.tag == 0 && e.last_call != ds->call_id) {
            slot = &e;
            break;
        }
        // a new tag for the same field buffer: its contents changed, so the stale copy is rebuilt
        // in place rather than kept beside a new one
        if (tag != 0 && e.tag != 0 && e.U == U && e.last_call != ds->call_id && !slot) slot = &e;
    }
    if (!slot) {
        // keep the cache small: at most 8 entries per device, evicting the
        // oldest entry this call has not handed out
        if (ds->gauge.size() >= 8) {
            for (auto it = ds->gauge.begin(); it != ds->gauge.end(); ++it)
                if ((*it)->last_call != ds->call_id) {
                    ds->gauge.erase(it);
                    break;
                }
        }
        std::unique_ptr<GaugeEntry> e(new GaugeEntry());
        e->g = g;
        e->dev.link_prec = link_p;
        e->dev.clover_prec = cl_p;
        size_t lb = (size_t)4 * 3 * g.V * unit_bytes(link_p);
        size_t cb = (size_t)18 * g.V * unit_bytes(cl_p);
        hipError_t h = hipMalloc(&e->dev.links, lb);
        if (h != hipSuccess) return hip_fail(h, "gauge links");
        h = hipMalloc(&e->dev.clover, cb);
        if (h != hipSuccess) return hip_fail(h, "clover");
        ds->gauge.emplace_back(std::move(e));
        slot = ds->gauge.back().get();
    }
    // (re)build: mark the slot unusable until validation passes
    slot->U = nullptr;
    slot->tag = 0;
    slot->eo.release();
    slot->dev.eo = &slot->eo;
    hipError_t h = ds->stats.ensure(256);
    if (h != hipSuccess) return hip_fail(h, "stats");
    unsigned* stats = (unsigned*)ds->stats.ptr;
    if ((h = hipMemsetAsync(stats, 0, 2 * sizeof(unsigned), st)) != hipSuccess) return hip_fail(h, "memset");
    if ((h = launch_link_ingest(g, link_p, U, slot->dev.links, stats, st)) != hipSuccess)
        return hip_fail(h, "link ingest");
    // an FP32 clover is the FP64 one rounded: converted from an FP64 copy of the same field,
    // parameters and tiling made or used in this call, else built
    const GaugeEntry* c64 = nullptr;
    if (cl_p == P_F32)
        for (auto& ep : ds->gauge) {
            const GaugeEntry& e = *ep;
            if (&e != slot && e.U == U && e.last_call == ds->call_id && e.dev.clover_prec == P_F64 &&
                e.kappa == kappa && e.csw == csw && std::memcmp(e.g.d, g.d, sizeof g.d) == 0 &&
                std::memcmp(e.g.lb, g.lb, sizeof g.lb) == 0) {
                c64 = &e;
                break;
            }
        }
    const double m4 = 1.0 / (2.0 * kappa);
    if (c64) {
        if ((h = launch_clover_to_f32(g, c64->dev.clover, slot->dev.clover, st)) != hipSuccess)
            return hip_fail(h, "clover conversion");
    } else if ((h = launch_clover_build(g, cl_p, U, m4, csw, slot->dev.clover, st)) != hipSuccess) {
        return hip_fail(h, "clover build");
    }
    unsigned host[2];
    if ((h = hipMemcpyAsync(host, stats, sizeof host, hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hip_fail(h, "stats copy");
    if ((h = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(h, "gauge ingest");
    if (host[1]) return fail(TM_ERR_NONFINITE, "gauge field holds NaN or Inf");
    float dev;
    std::memcpy(&dev, &host[0], sizeof dev);
    if (!(dev <= 1e-6f)) return fail(TM_ERR_NOT_SU3, "links deviate from SU(3) by %g (limit 1e-6)", (double)dev);
    slot->U = U;
    slot->tag = tag;
    slot->last_call = ds->call_id;
    slot->kappa = kappa;
    slot->csw = csw;
    *out = &slot->dev;
    return TM_OK;
}

// Internal spinor buffer carved from a workspace or wrapping caller memory.
SpinorBuf wrap_internal(void* base, const Geo& g, int nsys, Prec p) {
    SpinorBuf b;
    b.data = base;
    b.prec = p;
    b.nsys = nsys;
    b.scale = prec_has_scale(p)
                  ? reinterpret_cast<float*>(static_cast<char*>(base) + align256(spinor_data_bytes(g.V, nsys, p)))
                  : nullptr;
    return b;
}

size_t internal_bytes(const Geo& g, int nsys, Prec p) {
    return align256(spinor_data_bytes(g.V, nsys, p)) + align256(spinor_scale_bytes(g.V, nsys, p));
}

void fill_mu(const tm_geom* geom, double* mu) {
    for (int k = 0; k < kMaxSys; ++k) mu[k] = k < geom->nsys ? geom->mu[k] : 0.0;
}

// Inverse sets of one parity for the systems' |mu| values: built on first use
// and kept with the gauge entry; fills inv / sel / adj.
int prepare_site_inverses(const Geo& g, const GaugeDev& G, const double* mu, int nsys, int parity, hipStream_t st,
                          const void* inv[kMaxEoMu], unsigned char sel[kMaxSys], unsigned long long* adj) {
    if (g.lb[3] % 2 != 0)
        return fail(TM_ERR_BLOCKS, "even-odd solves need an even tile extent in x (got %d)", g.lb[3]);
    if (!G.eo) return fail(TM_ERR_ARG, "gauge entry without an even-odd cache");
    EoCache& c = *G.eo;
    double want[kMaxEoMu];
    int nwant = 0;
    *adj = 0;
    for (int k = 0; k < nsys; ++k) {
        const double am = std::fabs(mu[k]);
        int j = 0;
        while (j < nwant && want[j] != am) ++j;
        if (j == nwant) {
            if (nwant == kMaxEoMu)
                return fail(TM_ERR_ARG, "even-odd solves take at most %d distinct |mu| per call", kMaxEoMu);
            want[nwant++] = am;
        }
        sel[k] = (unsigned char)j;
        if (mu[k] < 0) *adj |= 1ull << k;
    }
    // keep the cache to the sets this call needs when it would overflow
    int missing = 0;
    for (int j = 0; j < nwant; ++j) {
        bool found = false;
        for (int i = 0; i < c.n; ++i) found |= c.absmu[i] == want[j] && c.parity[i] == parity;
        missing += !found;
    }
    if (c.n + missing > kMaxEoMu) c.release();
    for (int j = 0; j < nwant; ++j) {
        int i = 0;
        while (i < c.n && !(c.absmu[i] == want[j] && c.parity[i] == parity)) ++i;
        if (i == c.n) {
            void* p = nullptr;
            hipError_t h = hipMalloc(&p, eo_inverse_bytes(g, G.clover_prec));
            if (h != hipSuccess) return hip_fail(h, "even-odd inverses");
            if ((h = launch_eo_inverse(g, G.clover_prec, G.clover, want[j], parity, p, st)) != hipSuccess) {
                (void)hipFree(p);
                return hip_fail(h, "even-odd inverses");
            }
            c.absmu[c.n] = want[j];
            c.parity[c.n] = parity;
            c.inv[c.n] = p;
            ++c.n;
        }
        inv[j] = c.inv[i];
    }
    return TM_OK;
}

static int prepare_eo(const Geo& g, const GaugeDev& G, const double* mu, int nsys, hipStream_t st, SapArgs& a) {
    double mue[kMaxSys];  // the twist on the even sites, whose inverses the block solves use
    for (int k = 0; k < nsys; ++k) mue[k] = mu[k] + g.mu_shift[0];
    return prepare_site_inverses(g, G, mue, nsys, 0, st, a.eo_inv, a.eo_sel, &a.eo_adj);
}

int run_sap(const Geo& g, const GaugeDev& G, const SpinorBuf& b, const SpinorBuf& x, const double* mu, int nsys,
            int n_cycles, int mr_iters, bool x_zero, int sys_tile, hipStream_t st, bool eo, void* w_out) {
    if (w_out && !sap_fills_w(g, b.prec, G.link_prec, G.clover_prec, eo))
        return fail(TM_ERR_PREC, "D x from the half-sweep needs the 4^4 FP32 kernel with FP32 storage");
    SapArgs a;
    a.eo = eo ? 1 : 0;
    a.eo_adj = 0;
    for (int k = 0; k < kMaxEoMu; ++k) a.eo_inv[k] = nullptr;
    for (int k = 0; k < kMaxSys; ++k) a.eo_sel[k] = 0;
    if (eo) {
        int rc = prepare_eo(g, G, mu, nsys, st, a);
        if (rc) return rc;
    }
    a.g = g;
    a.links = G.links;
    a.clover = G.clover;
    a.b = b.data;
    a.b_scale = b.scale;
    a.x = x.data;
    a.x_scale = x.scale;
    a.nsys = nsys;
    a.sys_tile = sys_tile > 0 ? sys_tile : nsys;
    a.mr_iters = mr_iters;
    for (int k = 0; k < kMaxSys; ++k) a.mu[k] = mu[k];
    const Prec cp = b.prec == P_F64 ? P_F64 : P_F32;
    for (int cyc = 0; cyc < n_cycles; ++cyc)
        for (int colour = 0; colour < 2; ++colour) {
            a.colour = colour;
            // a zero guess: in the first cycle the swept colour's own x is
            // still zero, and before the first sweep the halo is zero too
            a.own_zero = (x_zero && cyc == 0) ? 1 : 0;
            a.halo_zero = (x_zero && cyc == 0 && colour == 0) ? 1 : 0;
            a.w_out = (cyc == n_cycles - 1 && colour == 1) ? w_out : nullptr;
            hipError_t h = launch_sap_half(a, b.prec, G.link_prec, G.clover_prec, cp, st);
            if (h == hipErrorInvalidConfiguration)
                return fail(TM_ERR_BLOCKS, "block of %d sites needs more LDS than the device has at this precision",
                            g.Vb);
            if (h != hipSuccess) return hip_fail(h, "sap half-sweep");
        }
    return TM_OK;
}

int run_dirac(const Geo& g, const GaugeDev& G, const SpinorBuf& in, const SpinorBuf& out, const double* mu, int nsys,
              Prec compute, hipStream_t st) {
    DiracArgs a;
    a.g = g;
    a.links = G.links;
    a.clover = G.clover;
    a.in = in.data;
    a.in_scale = in.scale;
    a.out = out.data;
    a.out_scale = out.scale;
    a.nsys = nsys;
    for (int k = 0; k < kMaxSys; ++k) a.mu[k] = mu[k];
    hipError_t h = launch_dirac(a, in.prec, out.prec, G.link_prec, G.clover_prec, compute, st);
    if (h == hipErrorInvalidValue) return fail(TM_ERR_PREC, "unsupported precision combination for the operator");
    if (h != hipSuccess) return hip_fail(h, "dirac");
    return TM_OK;
}

int run_dirac_colour(const Geo& g, const GaugeDev& G, const SpinorBuf& in, const SpinorBuf& out, const double* mu,
                     int nsys, int colour, hipStream_t st) {
    if (colour < 0 || colour > 1) return fail(TM_ERR_ARG, "colour must be 0 or 1");
    DiracArgs a;
    a.g = g;
    a.links = G.links;
    a.clover = G.clover;
    a.in = in.data;
    a.in_scale = in.scale;
    a.out = out.data;
    a.out_scale = out.scale;
    a.nsys = nsys;
    a.colour = colour;
    for (int k = 0; k < kMaxSys; ++k) a.mu[k] = mu[k];
    hipError_t h = launch_dirac_44(a, in.prec, out.prec, G.link_prec, G.clover_prec, st);
    if (h == hipErrorNotSupported) return fail(TM_ERR_PREC, "the operator on one colour needs the 4^4 FP32 tiles");
    if (h != hipSuccess) return hip_fail(h, "dirac on one colour");
    return TM_OK;
}

int check_sap_blocks(const tm_geom* geom, const int* block_dims, int tile[4]) {
    if (!block_dims) return fail(TM_ERR_ARG, "block_dims is NULL");
    for (int a = 0; a < 4; ++a) {
        if (block_dims[a] <= 0 || geom->dims[a] % block_dims[a] != 0)
            return fail(TM_ERR_DIMS, "block_dims[%d] = %d does not divide dims[%d] = %d", a, block_dims[a], a,
                        geom->dims[a]);
        if ((geom->dims[a] / block_dims[a]) % 2 != 0)
            return fail(TM_ERR_BLOCKS, "odd number of blocks (%d) along axis %d", geom->dims[a] / block_dims[a], a);
        tile[a] = block_dims[a];
    }
    if ((long long)tile[0] * tile[1] * tile[2] * tile[3] > 1024) return fail(TM_ERR_BLOCKS, "block holds more than 1024 sites");
    return TM_OK;
}

void drop_gauge(DeviceState* ds, const GaugeDev* G) {
    std::lock_guard<std::mutex> lock(ds->mutex);
    for (auto it = ds->gauge.begin(); it != ds->gauge.end(); ++it)
        if (&(*it)->dev == G) {
            ds->gauge.erase(it);
            return;
        }
}

bool gauge_held(DeviceState* ds, const GaugeDev* G) {
    std::lock_guard<std::mutex> lock(ds->mutex);
    for (auto& e : ds->gauge)
        if (&e->dev == G) return true;
    return false;
}

}  // namespace tmsap

using namespace tmsap;

extern "C" {

void tm_opts_default(tm_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->storage = TM_F64;
    o->compute = TM_F64;
    o->io = TM_IO_CANONICAL;
}

int tm_init(void) {
    int err = TM_OK;
    if (!device_state(&err)) return err;
    return noalloc_scratch(nullptr);
}

int tm_finalize(void) {
    std::lock_guard<std::mutex> lock(g_mutex);
    g_devices.clear();
    return TM_OK;
}

const char* tm_last_error(void) { return g_last_error.c_str(); }

int tm_gauge_release(const void* U) {
    std::lock_guard<std::mutex> lock(g_mutex);
    for (auto& d : g_devices) {
        std::lock_guard<std::mutex> l2(d->mutex);
        for (size_t i = 0; i < d->gauge.size();) {
            if (d->gauge[i]->U == U)
                d->gauge.erase(d->gauge.begin() + i);
            else
                ++i;
        }
    }
    return TM_OK;
}

size_t tm_spinor_bytes(const tm_geom* geom, const tm_opts* opts) {
    if (check_geom(geom) != TM_OK || check_opts(opts) != TM_OK) return 0;
    int tile[4];
    if (choose_tile(geom, opts->layout_block, tile) != TM_OK) return 0;
    Geo g = make_geo(geom, tile);
    return internal_bytes(g, geom->nsys, (Prec)opts->storage);
}

int tm_spinor_import(const tm_geom* geom, const void* canon, void* internal, const tm_opts* opts) {
    int rc;
    if ((rc = check_geom(geom)) || (rc = check_opts(opts))) return rc;
    if (!canon || !internal) return fail(TM_ERR_ARG, "null buffer");
    int tile[4];
    if ((rc = choose_tile(geom, opts->layout_block, tile))) return rc;
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    Geo g = make_geo(geom, tile);
    hipStream_t st = (hipStream_t)opts->stream;
    hipError_t h = ds->stats.ensure(256);
    if (h != hipSuccess) return hip_fail(h, "stats");
    SpinorBuf dst = wrap_internal(internal, g, geom->nsys, (Prec)opts->storage);
    if ((h = launch_spinor_import(g, dst, canon, (unsigned*)ds->stats.ptr + 2, st)) != hipSuccess)
        return hip_fail(h, "spinor import");
    return TM_OK;
}

int tm_spinor_export(const tm_geom* geom, const void* internal, void* canon, const tm_opts* opts) {
    int rc;
    if ((rc = check_geom(geom)) || (rc = check_opts(opts))) return rc;
    if (!canon || !internal) return fail(TM_ERR_ARG, "null buffer");
    int tile[4];
    if ((rc = choose_tile(geom, opts->layout_block, tile))) return rc;
    Geo g = make_geo(geom, tile);
    SpinorBuf src = wrap_internal(const_cast<void*>(internal), g, geom->nsys, (Prec)opts->storage);
    hipError_t h = launch_spinor_export(g, src, canon, (hipStream_t)opts->stream);
    if (h != hipSuccess) return hip_fail(h, "spinor export");
    return TM_OK;
}

// View of systems [first, first + count) of an internal buffer of geom->nsys systems.
static int internal_range(const tm_geom* geom, const void* internal, int first, int count, const tm_opts* opts,
                          Geo& g, SpinorBuf& view) {
    int rc;
    if ((rc = check_geom(geom)) || (rc = check_opts(opts))) return rc;
    if (!internal) return fail(TM_ERR_ARG, "null buffer");
    if (first < 0 || count < 1 || first + count > geom->nsys)
        return fail(TM_ERR_ARG, "systems %d..%d outside 0..%d", first, first + count - 1, geom->nsys - 1);
    int tile[4];
    if ((rc = choose_tile(geom, opts->layout_block, tile))) return rc;
    g = make_geo(geom, tile);
    const Prec p = (Prec)opts->storage;
    SpinorBuf all = wrap_internal(const_cast<void*>(internal), g, geom->nsys, p);
    view = all;
    view.data = static_cast<char*>(all.data) + (size_t)first * 6 * g.V * unit_bytes(p);
    view.scale = all.scale ? all.scale + (size_t)first * g.V : nullptr;
    view.nsys = count;
    return TM_OK;
}

int tm_spinor_import_range(const tm_geom* geom, const void* canon, void* internal, int first, int count,
                           const tm_opts* opts) {
    int rc;
    Geo g;
    SpinorBuf dst;
    if ((rc = internal_range(geom, internal, first, count, opts, g, dst))) return rc;
    if (!canon) return fail(TM_ERR_ARG, "null buffer");
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    hipError_t h = ds->stats.ensure(256);
    if (h != hipSuccess) return hip_fail(h, "stats");
    if ((h = launch_spinor_import(g, dst, canon, (unsigned*)ds->stats.ptr + 2, (hipStream_t)opts->stream)) !=
        hipSuccess)
        return hip_fail(h, "spinor import");
    return TM_OK;
}

int tm_spinor_export_range(const tm_geom* geom, const void* internal, void* canon, int first, int count,
                           const tm_opts* opts) {
    int rc;
    Geo g;
    SpinorBuf src;
    if ((rc = internal_range(geom, internal, first, count, opts, g, src))) return rc;
    if (!canon) return fail(TM_ERR_ARG, "null buffer");
    hipError_t h = launch_spinor_export(g, src, canon, (hipStream_t)opts->stream);
    if (h != hipSuccess) return hip_fail(h, "spinor export");
    return TM_OK;
}

int tm_dirac_apply(const tm_geom* geom, const void* U, const void* psi, void* out, double kappa, double c_sw,
                   const tm_opts* opts) {
    int rc;
    if ((rc = check_geom(geom)) || (rc = check_opts(opts))) return rc;
    if (!U || !psi || !out) return fail(TM_ERR_ARG, "null pointer");
    if (psi == out) return fail(TM_ERR_ARG, "psi and out alias");
    if (!(kappa > 0) || !std::isfinite(kappa) || !std::isfinite(c_sw)) return fail(TM_ERR_ARG, "bad kappa or c_sw");
    int tile[4];
    if ((rc = choose_tile(geom, opts->layout_block, tile))) return rc;
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    Geo g = make_geo(geom, tile);
    hipStream_t st = (hipStream_t)opts->stream;
    const Prec sp = (Prec)opts->storage, cp = (Prec)opts->compute;
    const GaugeDev* G;
    if ((rc = get_gauge(ds, g, U, kappa, c_sw, sp, opts->gauge_tag, st, &G))) return rc;
    double mu[kMaxSys];
    fill_mu(geom, mu);
    if (opts->io == TM_IO_INTERNAL) {
        SpinorBuf in = wrap_internal(const_cast<void*>(psi), g, geom->nsys, sp);
        SpinorBuf o = wrap_internal(out, g, geom->nsys, sp);
        return run_dirac(g, *G, in, o, mu, geom->nsys, cp, st);
    }
    size_t nb = internal_bytes(g, geom->nsys, sp);
    hipError_t h = ds->io.ensure(2 * nb);
    if (h != hipSuccess) return hip_fail(h, "workspace");
    hipError_t h2 = ds->stats.ensure(256);
    if (h2 != hipSuccess) return hip_fail(h2, "stats");
    SpinorBuf in = wrap_internal(ds->io.ptr, g, geom->nsys, sp);
    SpinorBuf o = wrap_internal(static_cast<char*>(ds->io.ptr) + nb, g, geom->nsys, sp);
    if ((h = launch_spinor_import(g, in, psi, (unsigned*)ds->stats.ptr + 2, st)) != hipSuccess)
        return hip_fail(h, "spinor import");
    if ((rc = run_dirac(g, *G, in, o, mu, geom->nsys, cp, st))) return rc;
    if ((h = launch_spinor_export(g, o, out, st)) != hipSuccess) return hip_fail(h, "spinor export");
    return TM_OK;
}

int tm_sap_smooth(const tm_geom* geom, const void* U, const void* b, void* x, double kappa, double c_sw,
                  const int block_dims[4], int n_cycles, int mr_iters, const tm_opts* opts) {
    int rc;
    if ((rc = check_geom(geom)) || (rc = check_opts(opts))) return rc;
    if (!U || !b || !x) return fail(TM_ERR_ARG, "null pointer");
    if (b == x) return fail(TM_ERR_ARG, "b and x alias");
    if (n_cycles < 0 || mr_iters < 0) return fail(TM_ERR_ARG, "negative cycle or MR count");
    if (!(kappa > 0) || !std::isfinite(kappa) || !std::isfinite(c_sw)) return fail(TM_ERR_ARG, "bad kappa or c_sw");
    int tile[4];
    if ((rc = check_sap_blocks(geom, block_dims, tile))) return rc;
    const Prec sp = (Prec)opts->storage;
    if (!sap_supported(sp, sp, clover_prec_for(sp), (Prec)opts->compute))
        return fail(TM_ERR_PREC, "unsupported precision combination for SAP");
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    Geo g = make_geo(geom, tile);
    hipStream_t st = (hipStream_t)opts->stream;
    const GaugeDev* G;
    if ((rc = get_gauge(ds, g, U, kappa, c_sw, sp, opts->gauge_tag, st, &G))) return rc;
    double mu[kMaxSys];
    fill_mu(geom, mu);
    if (opts->io == TM_IO_INTERNAL) {
        SpinorBuf bb = wrap_internal(const_cast<void*>(b), g, geom->nsys, sp);
        SpinorBuf xx = wrap_internal(x, g, geom->nsys, sp);
        return run_sap(g, *G, bb, xx, mu, geom->nsys, n_cycles, mr_iters, false, opts->sys_tile, st, opts->sap_eo);
    }
    size_t nb = internal_bytes(g, geom->nsys, sp);
    hipError_t h = ds->io.ensure(2 * nb);
    if (h != hipSuccess) return hip_fail(h, "workspace");
    if ((h = ds->stats.ensure(256)) != hipSuccess) return hip_fail(h, "stats");
    SpinorBuf bb = wrap_internal(ds->io.ptr, g, geom->nsys, sp);
    SpinorBuf xx = wrap_internal(static_cast<char*>(ds->io.ptr) + nb, g, geom->nsys, sp);
    if ((h = launch_spinor_import(g, bb, b, (unsigned*)ds->stats.ptr + 2, st)) != hipSuccess)
        return hip_fail(h, "spinor import");
    if ((h = launch_spinor_import(g, xx, x, (unsigned*)ds->stats.ptr + 2, st)) != hipSuccess)
        return hip_fail(h, "spinor import");
    if ((rc = run_sap(g, *G, bb, xx, mu, geom->nsys, n_cycles, mr_iters, false, opts->sys_tile, st, opts->sap_eo)))
        return rc;
    if ((h = launch_spinor_export(g, xx, x, st)) != hipSuccess) return hip_fail(h, "spinor export");
    return TM_OK;
}

}  // extern "C"
