// Two-level method (sections 2.2 - 2.6): setup, coarse GMRES, the
// preconditioner, and the C ABI of include/tm.h for them.
//
// The handle owns the basis P (N_v FP32 fields tiled by the aggregates) and
// the coarse stencil; workspaces grow on demand and stay with the handle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

#include "../../include/tm.h"
#include "tm_api_internal.h"
#include "tm_blas.h"
#include "tm_mg.h"

struct tm_mg {
    int device = 0;
    tm_geom geom{};    // dims, boundary phases and shifts of the setup (nsys 1, mu not kept)
    double mu0 = 0;    // twist of the setup
    double kappa = 0, csw = 0;
    const void* U = nullptr;
    unsigned long long tag = 0;
    tm_mg_params p{};
    tmsap::Geo g{};     // tile = aggregate
    long long nc = 0;   // coarse sites
    int n2 = 0;         // coarse components per site
    size_t field = 0;   // bytes of one FP32 field
    tmsap::DeviceBuffer P, Dc;
    tmsap::DeviceBuffer links, clover;  // own FP32 copy of the gauge data, tiled by the aggregates
    tmsap::GaugeDev gauge;
    tmsap::DeviceBuffer coarse;    // coarse vectors and the coarse Krylov basis
    tmsap::DeviceBuffer small;     // coefficients, norms, partial sums
    tmsap::DeviceBuffer fine;      // fine workspaces of setup and of the canonical entry points
    // even-odd coarse solver: inverses of the even-site blocks, one set per coarse twist,
    // valid until the stencil is rebuilt
    tmsap::DeviceBuffer inv[tmsap::kMgMaxInv];
    double inv_mu[tmsap::kMgMaxInv] = {};
    bool inv_ok[tmsap::kMgMaxInv] = {};
    unsigned long long inv_stamp[tmsap::kMgMaxInv] = {}, inv_clock = 0;
    double t_setup = 0;
    long long applications = 0, coarse_iters = 0;
    double t_coarse = 0;
};

namespace tmsap {

namespace {

typedef std::complex<double> zc;

int hc(hipError_t e, const char* where) { return e == hipSuccess ? TM_OK : hip_fail(e, where); }

// TM_VERBOSE=1: a progress line per setup iteration and per coarse solve on stderr.
bool verbose() {
    static int v = -1;
    if (v < 0) {
        const char* e = std::getenv("TM_VERBOSE");
        v = (e && e[0] && e[0] != '0') ? 1 : 0;
    }
    return v == 1;
}

MgArgs margs(const tm_mg* mg) {
    MgArgs m;
    m.g = mg->g;
    m.nv = mg->p.n_vec;
    m.P = mg->P.ptr;
    m.P_stride = mg->field;
    return m;
}

bool same_geometry(const tm_geom* a, const tm_geom* b) {
    for (int k = 0; k < 4; ++k)
        if (a->dims[k] != b->dims[k] || a->theta[k] != b->theta[k]) return false;
    return a->antiperiodic_t == b->antiperiodic_t && a->mu_shift[0] == b->mu_shift[0] &&
           a->mu_shift[1] == b->mu_shift[1];
}

int check_device(const tm_mg* mg) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != mg->device) return fail(TM_ERR_ARG, "the two-level handle lives on device %d, current is %d", mg->device, dev);
    return TM_OK;
}

// Small device arrays of one coarse solve over ns systems with restart m.
struct SmallBufs {
    double* mu;        // [ns]
    double2* h1;       // [ns][m + 1]
    double2* h2;       // [ns][m + 1]
    double* nrm;       // [ns]
    double* f;         // [ns]
    double2* y;        // [ns][m]
    double* partials;  // dots / norms
};

// partials sized for vectors of n complex entries
int carve_small(tm_mg* mg, int ns, int m, long long n, SmallBufs& s) {
    const size_t nblk = (size_t)mg_blas_blocks(n);
    const size_t doubles = 3 * (size_t)ns + 2 * 2 * (size_t)ns * (m + 1) + 2 * (size_t)ns * m +
                           (size_t)ns * 32 * nblk + 64;
    hipError_t e = mg->small.ensure(doubles * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "two-level scratch");
    double* p = static_cast<double*>(mg->small.ptr);
    s.mu = p; p += ns;
    s.nrm = p; p += ns;
    s.f = p; p += ns;
    s.h1 = reinterpret_cast<double2*>(p); p += 2 * (size_t)ns * (m + 1);
    s.h2 = reinterpret_cast<double2*>(p); p += 2 * (size_t)ns * (m + 1);
    s.y = reinterpret_cast<double2*>(p); p += 2 * (size_t)ns * m;
    s.partials = p;
    return TM_OK;
}

constexpr int kChunk = 16;  // basis vectors per dot / axpy pass (mg_blas limit)

// w_s -= V h_s over basis vectors 0..nv-1 (coefficients from h, stride hs).
int basis_axpy(const float2* V, size_t vstride, int nv, const double2* h, int hs, double sign, float2* w,
               size_t sstride, int ns, long long n, hipStream_t st) {
    for (int i0 = 0; i0 < nv; i0 += kChunk) {
        const int cnt = std::min(kChunk, nv - i0);
        hipError_t e = mg_blas_axpy(V + (size_t)i0 * vstride, vstride, cnt, h + i0, hs, sign, w, sstride, ns, n, st);
        if (e != hipSuccess) return hip_fail(e, "coarse axpy");
    }
    return TM_OK;
}

int basis_dots(const float2* V, size_t vstride, int nv, const float2* w, size_t sstride, int ns, long long n,
               double* partials, double2* out, int os, hipStream_t st) {
    for (int i0 = 0; i0 < nv; i0 += kChunk) {
        const int cnt = std::min(kChunk, nv - i0);
        hipError_t e = mg_blas_dots(V + (size_t)i0 * vstride, vstride, cnt, w, sstride, ns, n, partials, out + i0, os, st);
        if (e != hipSuccess) return hip_fail(e, "coarse dots");
    }
    return TM_OK;
}

// y = A x for the ns systems of one coarse solve (full coarse vectors)
typedef std::function<int(const float2* x, float2* y)> CoarseOp;

// Host copy of ||v_s|| for ns coarse vectors.
int coarse_norms(tm_mg* mg, const float2* v, int ns, const SmallBufs& sb, double* out, hipStream_t st) {
    const long long n = mg->nc * mg->n2;
    int rc;
    if ((rc = hc(mg_blas_norm2(v, (size_t)n, ns, n, sb.partials, sb.nrm, st), "norm"))) return rc;
    if ((rc = hc(hipMemcpyAsync(out, sb.nrm, ns * sizeof(double), hipMemcpyDeviceToHost, st), "copy"))) return rc;
    if ((rc = hc(hipStreamSynchronize(st), "coarse solve"))) return rc;
    for (int k = 0; k < ns; ++k) out[k] = std::sqrt(std::max(0.0, out[k]));
    return TM_OK;
}

// GMRES(m) for A x = b over ns systems from x = 0; b and x [ns][nc][n2] FP32 (x
// overwritten).  A system stops when its residual estimate is <= tol * bref[s]
// (tol 0: never).  work holds (m + 2) ns coarse vectors (the basis and one more).
// Classical Gram-Schmidt applied twice; the host solves the small least-squares
// problems.  Returns the largest number of steps any system took in *iters.
int gmres_core(tm_mg* mg, int ns, const CoarseOp& A, const double* bref, const float2* b, float2* x, float2* work,
               double tol, int m, int maxr, const SmallBufs& sb, int* iters, hipStream_t st) {
    const long long n = mg->nc * mg->n2;
    const size_t vs = (size_t)n, vstride = (size_t)ns * n;
    int rc;
    float2* V = work;
    float2* w = V + (size_t)(m + 1) * vstride;
    std::vector<double> host(2 * 2 * (size_t)ns * (m + 1) + 4 * (size_t)ns);
    if ((rc = hc(blas_zero(x, (size_t)ns * n * sizeof(float2), st), "zero"))) return rc;
    std::vector<double> bn(bref, bref + ns), beta(ns), fh(ns);
    std::vector<zc> H((size_t)ns * (m + 1) * m), sn((size_t)ns * m), gv((size_t)ns * (m + 1));
    std::vector<double> cs((size_t)ns * m);
    std::vector<int> kdim(ns);
    std::vector<char> frozen(ns);
    int steps_max = 0;
    for (int cyc = 0; cyc < maxr; ++cyc) {
        // v0 = b - A x (b itself in the first cycle)
        if (cyc == 0) {
            for (int k = 0; k < ns; ++k) host[k] = 1.0;
            if ((rc = hc(hipMemcpyAsync(sb.f, host.data(), ns * sizeof(double), hipMemcpyHostToDevice, st), "copy")))
                return rc;
            if ((rc = hc(mg_blas_scale(b, sb.f, V, vs, ns, n, st), "copy"))) return rc;
        } else {
            if ((rc = A(x, V))) return rc;
            if ((rc = hc(mg_blas_sub_from(b, V, vs, ns, n, st), "residual"))) return rc;
        }
        if ((rc = hc(mg_blas_norm2(V, vs, ns, n, sb.partials, sb.nrm, st), "norm"))) return rc;
        if ((rc = hc(hipMemcpyAsync(host.data(), sb.nrm, ns * sizeof(double), hipMemcpyDeviceToHost, st), "copy")))
            return rc;
        if ((rc = hc(hipStreamSynchronize(st), "coarse solve"))) return rc;
        bool any = false;
        for (int k = 0; k < ns; ++k) {
            beta[k] = std::sqrt(std::max(0.0, host[k]));
            if (!std::isfinite(beta[k])) return fail(TM_ERR_NONFINITE, "non-finite coarse residual (system %d)", k);
            frozen[k] = beta[k] == 0.0 || (tol > 0 && beta[k] <= tol * bn[k]);
            any |= !frozen[k];
            fh[k] = frozen[k] ? 0.0 : 1.0 / beta[k];
            for (int i = 0; i <= m; ++i) gv[(size_t)k * (m + 1) + i] = 0.0;
            gv[(size_t)k * (m + 1)] = frozen[k] ? 0.0 : beta[k];
            kdim[k] = 0;
        }
        if (!any) break;
        if ((rc = hc(hipMemcpyAsync(sb.f, fh.data(), ns * sizeof(double), hipMemcpyHostToDevice, st), "copy"))) return rc;
        if ((rc = hc(mg_blas_scale(V, sb.f, V, vs, ns, n, st), "scale"))) return rc;
        int jdone = 0;
        for (int j = 0; j < m; ++j) {
            float2* vj = V + (size_t)j * vstride;
            if ((rc = A(vj, w))) return rc;
            const int nb = j + 1;
            if ((rc = basis_dots(V, vstride, nb, w, vs, ns, n, sb.partials, sb.h1, m + 1, st))) return rc;
            if ((rc = basis_axpy(V, vstride, nb, sb.h1, m + 1, -1.0, w, vs, ns, n, st))) return rc;
            if ((rc = basis_dots(V, vstride, nb, w, vs, ns, n, sb.partials, sb.h2, m + 1, st))) return rc;
            if ((rc = basis_axpy(V, vstride, nb, sb.h2, m + 1, -1.0, w, vs, ns, n, st))) return rc;
            if ((rc = hc(mg_blas_norm2(w, vs, ns, n, sb.partials, sb.nrm, st), "norm"))) return rc;
            double* hh1 = host.data();
            double* hh2 = hh1 + 2 * (size_t)ns * (m + 1);
            double* hn2 = hh2 + 2 * (size_t)ns * (m + 1);
            if ((rc = hc(hipMemcpyAsync(hh1, sb.h1, 2 * (size_t)ns * (m + 1) * sizeof(double), hipMemcpyDeviceToHost, st),
                         "copy")))
                return rc;
            if ((rc = hc(hipMemcpyAsync(hh2, sb.h2, 2 * (size_t)ns * (m + 1) * sizeof(double), hipMemcpyDeviceToHost, st),
                         "copy")))
                return rc;
            if ((rc = hc(hipMemcpyAsync(hn2, sb.nrm, ns * sizeof(double), hipMemcpyDeviceToHost, st), "copy"))) return rc;
            if ((rc = hc(hipStreamSynchronize(st), "coarse Arnoldi step"))) return rc;
            bool all_frozen = true;
            for (int k = 0; k < ns; ++k) {
                fh[k] = 0.0;
                if (frozen[k]) continue;
                zc* Hk = &H[(size_t)k * (m + 1) * m];
                for (int i = 0; i < nb; ++i) {
                    const double* a = hh1 + ((size_t)k * (m + 1) + i) * 2;
                    const double* c2 = hh2 + ((size_t)k * (m + 1) + i) * 2;
                    Hk[i * m + j] = zc(a[0] + c2[0], a[1] + c2[1]);
                }
                const double hn = std::sqrt(std::max(0.0, hn2[k]));
                if (!std::isfinite(hn)) return fail(TM_ERR_NONFINITE, "non-finite coarse Arnoldi step (system %d)", k);
                Hk[(j + 1) * m + j] = hn;
                fh[k] = hn > 0 ? 1.0 / hn : 0.0;
                double* csk = &cs[(size_t)k * m];
                zc* snk = &sn[(size_t)k * m];
                zc* gk = &gv[(size_t)k * (m + 1)];
                for (int i = 0; i < j; ++i) {
                    const zc a = Hk[i * m + j], c2 = Hk[(i + 1) * m + j];
                    Hk[i * m + j] = csk[i] * a + snk[i] * c2;
                    Hk[(i + 1) * m + j] = -std::conj(snk[i]) * a + csk[i] * c2;
                }
                const zc a = Hk[j * m + j], c2 = Hk[(j + 1) * m + j];
                const double t = std::sqrt(std::norm(a) + std::norm(c2));
                if (std::abs(a) == 0.0) {
                    csk[j] = 0.0;
                    snk[j] = 1.0;
                } else {
                    csk[j] = std::abs(a) / t;
                    snk[j] = (a / std::abs(a)) * std::conj(c2) / t;
                }
                Hk[j * m + j] = csk[j] * a + snk[j] * c2;
                Hk[(j + 1) * m + j] = 0.0;
                gk[j + 1] = -std::conj(snk[j]) * gk[j];
                gk[j] = csk[j] * gk[j];
                kdim[k] = j + 1;
                if ((tol > 0 && std::abs(gk[j + 1]) <= tol * bn[k]) || hn == 0.0) {
                    frozen[k] = 1;
                    fh[k] = 0.0;
                }
                all_frozen &= (bool)frozen[k];
            }
            jdone = j + 1;
            ++steps_max;
            if (all_frozen || j + 1 == m) break;
            if ((rc = hc(hipMemcpyAsync(sb.f, fh.data(), ns * sizeof(double), hipMemcpyHostToDevice, st), "copy")))
                return rc;
            if ((rc = hc(mg_blas_scale(w, sb.f, V + (size_t)(j + 1) * vstride, vs, ns, n, st), "scale"))) return rc;
        }
        // x += V y per system (zero beyond its Krylov dimension)
        std::vector<double> yh(2 * (size_t)ns * m, 0.0);
        for (int k = 0; k < ns; ++k) {
            const zc* Hk = &H[(size_t)k * (m + 1) * m];
            const zc* gk = &gv[(size_t)k * (m + 1)];
            std::vector<zc> y(kdim[k]);
            for (int i = kdim[k] - 1; i >= 0; --i) {
                zc t = gk[i];
                for (int q = i + 1; q < kdim[k]; ++q) t -= Hk[i * m + q] * y[q];
                y[i] = t / Hk[i * m + i];
            }
            for (int i = 0; i < kdim[k]; ++i) {
                yh[((size_t)k * m + i) * 2] = y[i].real();
                yh[((size_t)k * m + i) * 2 + 1] = y[i].imag();
            }
        }
        if (jdone > 0) {
            if ((rc = hc(hipMemcpyAsync(sb.y, yh.data(), yh.size() * sizeof(double), hipMemcpyHostToDevice, st), "copy")))
                return rc;
            if ((rc = basis_axpy(V, vstride, jdone, sb.y, m, 1.0, x, vs, ns, n, st))) return rc;
            // the host vector yh must outlive the copy
            if ((rc = hc(hipStreamSynchronize(st), "coarse update"))) return rc;
        }
        bool all = true;
        for (int k = 0; k < ns; ++k) all &= (bool)frozen[k];
        if (all && tol > 0) break;
    }
    if (iters) *iters = steps_max;
    return TM_OK;
}


// Coarse floats a solve over ns systems with restart m needs after the caller's two
// vectors c, e: the basis, w, and for the even-odd solver three more.
size_t coarse_work_vectors(const tm_mg* mg, int m) { return (size_t)m + 2 + (mg->p.coarse_eo ? 3 : 0); }

// Even-site block inverses for the twists mu_c[0..ns) (at most kMgMaxInv distinct):
// cached sets are reused, missing ones computed; fills a.sets and a.sel.
int ensure_inverses(tm_mg* mg, int ns, const double* mu_c, BlockMulArgs& a, hipStream_t st) {
    bool used[kMgMaxInv] = {};
    const int n2 = mg->n2;
    for (int s = 0; s < ns; ++s) {
        int k = 0;
        while (k < kMgMaxInv && !(mg->inv_ok[k] && mg->inv_mu[k] == mu_c[s])) ++k;
        if (k == kMgMaxInv) {  // a set not needed by this call: an empty one, else the least recently used
            k = -1;
            for (int q = 0; q < kMgMaxInv; ++q) {
                if (used[q]) continue;
                if (k < 0 || (!mg->inv_ok[q] && mg->inv_ok[k]) ||
                    (mg->inv_ok[q] == mg->inv_ok[k] && mg->inv_stamp[q] < mg->inv_stamp[k]))
                    k = q;
            }
            if (k < 0) return fail(TM_ERR_ARG, "more than %d distinct coarse twists in one coarse solve", kMgMaxInv);
            hipError_t e = mg->inv[k].ensure((size_t)(mg->nc / 2) * n2 * n2 * sizeof(float2));
            if (e != hipSuccess) return hip_fail(e, "coarse block inverses");
            mg->inv_ok[k] = false;
            int rc;
            if ((rc = hc(launch_mg_block_inverse(mg->g, mg->p.n_vec, (const float2*)mg->Dc.ptr, mu_c[s], 0,
                                                 static_cast<float2*>(mg->inv[k].ptr), st),
                         "coarse block inverses")))
                return rc;
            mg->inv_ok[k] = true;
            mg->inv_mu[k] = mu_c[s];
        }
        used[k] = true;
        mg->inv_stamp[k] = ++mg->inv_clock;
        a.sets[k] = static_cast<const float2*>(mg->inv[k].ptr);
        a.sel[s] = (unsigned char)k;
    }
    return TM_OK;
}

// Even-odd preconditioned GMRES on the coarse grid (section 2.5's reduction, used as
// the coarsest-grid solver in Table 1): GMRES(m) for the odd-site system
// (D_oo - D_oe D_ee^-1 D_eo) x_o = b_o - D_oe D_ee^-1 b_e, then
// x_e = D_ee^-1 (b_e - D_eo x_o).  The full residual's even part vanishes and its odd
// part is the reduced residual, so the stop compares with tol ||b||.  Vectors keep the
// full coarse layout with zero even parts; at most kMgMaxInv distinct twists.
int coarse_gmres_eo(tm_mg* mg, int ns, const double* mu_c, const float2* b, float2* x, float2* work, double tol, int m,
                    int maxr, int* iters, hipStream_t st) {
    const long long n = mg->nc * mg->n2;
    const Geo& g = mg->g;
    const int nv = mg->p.n_vec;
    const float2* Dc = static_cast<const float2*>(mg->Dc.ptr);
    int rc;
    BlockMulArgs a{};
    a.g = g;
    a.nv = nv;
    a.nsys = ns;
    a.parity = 0;
    a.zero_other = false;
    if ((rc = ensure_inverses(mg, ns, mu_c, a, st))) return rc;
    SmallBufs sb;
    if ((rc = carve_small(mg, ns, m, n, sb))) return rc;
    if ((rc = hc(hipMemcpyAsync(sb.mu, mu_c, ns * sizeof(double), hipMemcpyHostToDevice, st), "copy"))) return rc;
    float2* t = work + (size_t)(m + 2) * ns * n;
    float2* u = t + (size_t)ns * n;
    float2* bh = u + (size_t)ns * n;
    std::vector<double> bref(ns);
    if ((rc = coarse_norms(mg, b, ns, sb, bref.data(), st))) return rc;
    // bh_o = b_o - D_oe D_ee^-1 b_e, bh_e = 0
    a.x = b;
    a.y = u;
    if ((rc = hc(launch_mg_block_mul(a, st), "coarse block inverses"))) return rc;
    if ((rc = hc(launch_mg_coarse_part(g, nv, Dc, nullptr, nullptr, u, -1.0, b, 1, true, bh, ns, st), "coarse operator")))
        return rc;
    const CoarseOp dhat = [&](const float2* in, float2* out) -> int {
        int r;
        // t_e = D_eo in_o; u_e = D_ee^-1 t_e; out_o = D_oo in_o - D_oe u_e, out_e = 0
        if ((r = hc(launch_mg_coarse_part(g, nv, Dc, nullptr, nullptr, in, 1.0, nullptr, 0, false, t, ns, st),
                    "coarse operator")))
            return r;
        BlockMulArgs am = a;
        am.x = t;
        am.y = u;
        if ((r = hc(launch_mg_block_mul(am, st), "coarse block inverses"))) return r;
        return hc(launch_mg_coarse_part(g, nv, Dc, sb.mu, in, u, -1.0, nullptr, 1, true, out, ns, st), "coarse operator");
    };
    if ((rc = gmres_core(mg, ns, dhat, bref.data(), bh, x, work, tol, m, maxr, sb, iters, st))) return rc;
    // x_e = D_ee^-1 (b_e - D_eo x_o)
    if ((rc = hc(launch_mg_coarse_part(g, nv, Dc, nullptr, nullptr, x, -1.0, b, 0, false, t, ns, st), "coarse operator")))
        return rc;
    a.x = t;
    a.y = x;
    return hc(launch_mg_block_mul(a, st), "coarse block inverses");
}

}  // namespace

// Solves (D_c + i mu_c[s] Gamma5c) x_s = b_s for ns systems (b, x [ns][nc][n2] FP32,
// x overwritten; mu_c host [ns]) by GMRES(m) on the full coarse operator or, when the
// handle's coarse_eo is set, on the even-odd reduced one.  The workspace sits in the
// handle's coarse buffer after 2 ns coarse vectors left to the caller.  Returns the
// largest number of GMRES steps any system took in *iters.
int mg_coarse_gmres(tm_mg* mg, int ns, const double* mu_c, const float2* b, float2* x, double tol, int m, int maxr,
                    int* iters, hipStream_t st) {
    const long long n = mg->nc * mg->n2;
    int rc;
    hipError_t e = mg->coarse.ensure((2 + coarse_work_vectors(mg, m)) * (size_t)ns * n * sizeof(float2));
    if (e != hipSuccess) return hip_fail(e, "coarse Krylov basis");
    float2* work = static_cast<float2*>(mg->coarse.ptr) + 2 * (size_t)ns * n;
    if (mg->p.coarse_eo) {
        // systems in runs of at most kMgMaxInv distinct twists
        int most = 0;
        for (int s0 = 0; s0 < ns;) {
            std::vector<double> seen;
            int s1 = s0;
            while (s1 < ns) {
                if (std::find(seen.begin(), seen.end(), mu_c[s1]) == seen.end()) {
                    if ((int)seen.size() == kMgMaxInv) break;
                    seen.push_back(mu_c[s1]);
                }
                ++s1;
            }
            int it = 0;
            if ((rc = coarse_gmres_eo(mg, s1 - s0, mu_c + s0, b + (size_t)s0 * n, x + (size_t)s0 * n, work, tol, m, maxr,
                                      &it, st)))
                return rc;
            most = std::max(most, it);
            s0 = s1;
        }
        if (iters) *iters = most;
        return TM_OK;
    }
    SmallBufs sb;
    if ((rc = carve_small(mg, ns, m, n, sb))) return rc;
    if ((rc = hc(hipMemcpyAsync(sb.mu, mu_c, ns * sizeof(double), hipMemcpyHostToDevice, st), "copy"))) return rc;
    std::vector<double> bref(ns);
    if ((rc = coarse_norms(mg, b, ns, sb, bref.data(), st))) return rc;
    const Geo g = mg->g;
    const int nv = mg->p.n_vec;
    const float2* Dc = static_cast<const float2*>(mg->Dc.ptr);
    const double* mud = sb.mu;
    const CoarseOp full = [&](const float2* in, float2* out) -> int {
        return hc(launch_mg_coarse_apply(g, nv, Dc, mud, in, out, ns, st), "coarse operator");
    };
    return gmres_core(mg, ns, full, bref.data(), b, x, work, tol, m, maxr, sb, iters, st);
}

// The two-level preconditioner on internal FP32 fields (tiled by the
// aggregates): z = P D_c^-1 P^+ r, then post_cycles SAP cycles from z.
int mg_apply(tm_mg* mg, DeviceState* ds, const SpinorBuf& r, const SpinorBuf& z, const double* mu, int ns,
             hipStream_t st) {
    (void)ds;
    int rc;
    const long long n = mg->nc * mg->n2;
    const int m = mg->p.coarse_restart;
    hipError_t e = mg->coarse.ensure((2 + coarse_work_vectors(mg, m)) * (size_t)ns * n * sizeof(float2));
    if (e != hipSuccess) return hip_fail(e, "coarse vectors");
    float2* c = static_cast<float2*>(mg->coarse.ptr);
    float2* ec = c + (size_t)ns * n;
    const MgArgs ma = margs(mg);
    const size_t fb = internal_bytes(mg->g, 1, P_F32);
    if ((rc = hc(launch_mg_restrict(ma, r.data, fb, ns, c, 0, (size_t)n, (size_t)mg->n2, st), "restriction"))) return rc;
    std::vector<double> muc(ns);
    for (int k = 0; k < ns; ++k) muc[k] = mg->p.delta * mu[k];
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    if (timed) (void)hipEventRecord(e0, st);
    int it = 0;
    rc = mg_coarse_gmres(mg, ns, muc.data(), c, ec, mg->p.coarse_tol, m, mg->p.coarse_max_restarts, &it, st);
    if (timed) {
        (void)hipEventRecord(e1, st);
        float ms = 0;
        if (rc == TM_OK && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            mg->t_coarse += ms * 1e-3;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc) return rc;
    mg->applications += 1;
    mg->coarse_iters += it;
    if (verbose()) {
        std::fprintf(stderr, "[tm] two-level: coarse GMRES %d steps for %d systems, coarse time so far %.3f s\n", it, ns,
                     mg->t_coarse);
        std::fflush(stderr);
    }
    if ((rc = hc(launch_mg_prolong(ma, ec, ns, z.data, fb, st), "prolongation"))) return rc;
    if (mg->p.post_cycles > 0)
        return run_sap(mg->g, mg->gauge, r, z, mu, ns, mg->p.post_cycles, mg->p.mr_iters, false, 0, st);
    return TM_OK;
}

namespace {

// Orthonormalises nv FP32 fields over the whole lattice, in order: block classical
// Gram-Schmidt twice, in panels of 4 fields (each pass reads the earlier fields once
// for the whole panel), then classical Gram-Schmidt twice inside the panel.  Same
// result as Gram-Schmidt vector by vector, up to rounding.
int orthonormalize_fields(tm_mg* mg, float2* v, int nv, hipStream_t st) {
    constexpr int kPb = 4, kPd = 4, kPa = 8;  // panel width, basis vectors per dot / axpy pass
    const long long n = 12 * mg->g.V;  // complex entries of one field
    const size_t fs = mg->field / sizeof(float2);
    SmallBufs sb;
    int rc;
    if ((rc = carve_small(mg, kPb, kMgMaxVec, n, sb))) return rc;
    const int hs = kMgMaxVec + 1;  // coefficient stride per panel vector
    for (int p0 = 0; p0 < nv; p0 += kPb) {
        const int pb = std::min(kPb, nv - p0);
        float2* W = v + (size_t)p0 * fs;
        for (int pass = 0; pass < 2 && p0 > 0; ++pass) {
            for (int i0 = 0; i0 < p0; i0 += kPd)
                if ((rc = hc(mg_blas_panel_dots(v + (size_t)i0 * fs, fs, std::min(kPd, p0 - i0), W, fs, pb, n,
                                                sb.partials, sb.h1 + i0, hs, st),
                             "panel dots")))
                    return rc;
            for (int i0 = 0; i0 < p0; i0 += kPa)
                if ((rc = hc(mg_blas_panel_axpy(v + (size_t)i0 * fs, fs, std::min(kPa, p0 - i0), sb.h1 + i0, hs, W,
                                                fs, pb, n, st),
                             "panel update")))
                    return rc;
        }
        for (int i = p0; i < p0 + pb; ++i) {
            float2* vi = v + (size_t)i * fs;
            if (i > p0) {
                for (int pass = 0; pass < 2; ++pass) {
                    if ((rc = basis_dots(W, fs, i - p0, vi, 0, 1, n, sb.partials, sb.h1, 0, st))) return rc;
                    if ((rc = basis_axpy(W, fs, i - p0, sb.h1, 0, -1.0, vi, 0, 1, n, st))) return rc;
                }
            }
            if ((rc = hc(mg_blas_norm2(vi, 0, 1, n, sb.partials, sb.nrm, st), "norm"))) return rc;
            double n2 = 0;
            if ((rc = hc(hipMemcpyAsync(&n2, sb.nrm, sizeof(double), hipMemcpyDeviceToHost, st), "copy"))) return rc;
            if ((rc = hc(hipStreamSynchronize(st), "orthonormalisation"))) return rc;
            if (!std::isfinite(n2)) return fail(TM_ERR_NONFINITE, "non-finite test vector %d", i);
            const double f = n2 > 0 ? 1.0 / std::sqrt(n2) : 0.0;
            if ((rc = hc(hipMemcpyAsync(sb.f, &f, sizeof(double), hipMemcpyHostToDevice, st), "copy"))) return rc;
            if ((rc = hc(mg_blas_scale(vi, sb.f, vi, 0, 1, n, st), "scale"))) return rc;
            if ((rc = hc(hipStreamSynchronize(st), "orthonormalisation"))) return rc;
        }
    }
    return TM_OK;
}

// P = aggregate-wise orthonormalised copy of the fields v; then the stencil.
int build_coarse(tm_mg* mg, const GaugeDev& G, const void* v, void* W, int chunk, hipStream_t st) {
    int rc;
    const int nv = mg->p.n_vec, n2 = mg->n2;
    if ((rc = hc(hipMemcpyAsync(mg->P.ptr, v, (size_t)nv * mg->field, hipMemcpyDeviceToDevice, st), "copy"))) return rc;
    const MgArgs ma = margs(mg);
    for (int k = 0; k < kMgMaxInv; ++k) mg->inv_ok[k] = false;  // the block inverses follow the stencil
    if ((rc = hc(launch_mg_block_orthonormalize(ma, mg->P.ptr, st), "aggregate orthonormalisation"))) return rc;
    const size_t fb = internal_bytes(mg->g, 1, P_F32);
    for (int t = 0; t < 9; ++t)
        for (int b0 = 0; b0 < n2; b0 += chunk) {
            const int nb = std::min(chunk, n2 - b0);
            if ((rc = hc(launch_mg_term(ma, G.links, G.clover, t, b0, nb, W, fb, st), "coarse stencil terms"))) return rc;
            if ((rc = hc(launch_mg_restrict(ma, W, fb, nb, static_cast<float2*>(mg->Dc.ptr),
                                            (size_t)t * n2 * n2 + (size_t)b0 * n2, (size_t)n2, (size_t)9 * n2 * n2, st),
                         "coarse stencil")))
                return rc;
        }
    return TM_OK;
}

int check_params(const tm_geom* geom, const tm_mg_params* p, int tile[4]) {
    if (!p) return fail(TM_ERR_ARG, "params is NULL");
    if (p->n_vec < 1 || p->n_vec > kMgMaxVec) return fail(TM_ERR_ARG, "n_vec = %d outside 1..%d", p->n_vec, kMgMaxVec);
    if (p->setup_iters < 0 || p->setup_cycles < 0 || p->post_cycles < 0 || p->mr_iters < 0)
        return fail(TM_ERR_ARG, "negative setup, cycle or MR count");
    if (p->coarse_restart < 1 || p->coarse_restart > 128 || p->coarse_max_restarts < 1)
        return fail(TM_ERR_ARG, "coarse_restart must be 1..128 and coarse_max_restarts >= 1");
    if (!(p->delta > 0) || !std::isfinite(p->delta) || !(p->coarse_tol >= 0) || !std::isfinite(p->coarse_tol))
        return fail(TM_ERR_ARG, "bad delta or coarse_tol");
    if (p->coarse_eo != 0 && p->coarse_eo != 1) return fail(TM_ERR_ARG, "coarse_eo must be 0 or 1");
    return check_sap_blocks(geom, p->block_dims, tile);
}

int check_storage(const tm_opts* opts) {
    if (opts->storage != TM_F32) return fail(TM_ERR_PREC, "the two-level method runs at FP32 storage");
    return TM_OK;
}

}  // namespace

int mg_matches(const tm_mg* mg, const tm_geom* geom) {
    if (!same_geometry(&mg->geom, geom))
        return fail(TM_ERR_ARG, "geometry differs from the two-level handle's (dims, boundary phases or mu shifts)");
    return check_device(mg);
}

size_t mg_workspace_held(const tm_mg* mg) {
    size_t b = mg->coarse.bytes + mg->small.bytes;
    for (int k = 0; k < kMgMaxInv; ++k) b += mg->inv[k].bytes;
    return b;
}

size_t mg_workspace_per_sys(const tm_mg* mg) {
    return (2 + coarse_work_vectors(mg, mg->p.coarse_restart)) * mg->nc * mg->n2 * sizeof(float2);
}

void mg_block_dims(const tm_mg* mg, int bd[4]) {
    for (int a = 0; a < 4; ++a) bd[a] = mg->p.block_dims[a];
}

}  // namespace tmsap

using namespace tmsap;

extern "C" {

void tm_mg_params_default(tm_mg_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    for (int a = 0; a < 4; ++a) p->block_dims[a] = 4;
    p->n_vec = 28;
    p->setup_iters = 5;
    p->setup_cycles = 4;
    p->delta = 5.2;
    p->coarse_tol = 0.1;
    p->coarse_restart = 100;
    p->coarse_max_restarts = 5;
    p->post_cycles = 4;
    p->mr_iters = 3;
    p->coarse_eo = 1;
}

int tm_mg_setup(const tm_geom* geom, const void* U, double kappa, double c_sw, const tm_mg_params* params,
                const void* v0, tm_mg** out, const tm_opts* opts) {
    int rc;
    if (!out) return fail(TM_ERR_ARG, "mg is NULL");
    *out = nullptr;
    if ((rc = check_geom(geom)) || (rc = check_opts(opts)) || (rc = check_storage(opts))) return rc;
    if (geom->nsys != 1) return fail(TM_ERR_ARG, "the setup takes one twist (nsys = 1), got nsys = %d", geom->nsys);
    if (!U || !v0) return fail(TM_ERR_ARG, "null pointer");
    if (!(kappa > 0) || !std::isfinite(kappa) || !std::isfinite(c_sw)) return fail(TM_ERR_ARG, "bad kappa or c_sw");
    int tile[4];
    if ((rc = check_params(geom, params, tile))) return rc;
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)opts->stream;
    std::unique_ptr<tm_mg> mg(new tm_mg());
    if ((rc = hc(hipGetDevice(&mg->device), "hipGetDevice"))) return rc;
    mg->geom = *geom;
    mg->geom.mu = nullptr;
    mg->mu0 = geom->mu[0];
    mg->kappa = kappa;
    mg->csw = c_sw;
    mg->U = U;
    mg->tag = opts->gauge_tag;
    mg->p = *params;
    mg->g = make_geo(geom, tile);
    mg->nc = mg->g.V / mg->g.Vb;
    mg->n2 = 2 * params->n_vec;
    mg->field = internal_bytes(mg->g, 1, P_F32);
    const int nv = params->n_vec;
    const GaugeDev* Gc;
    if ((rc = get_gauge(ds, mg->g, U, kappa, c_sw, P_F32, opts->gauge_tag, st, &Gc))) return rc;
    hipError_t e;
    // the handle keeps its own copy of the links and the clover term
    const size_t lbytes = (size_t)4 * 3 * mg->g.V * unit_bytes(P_F32), cbytes = (size_t)18 * mg->g.V * unit_bytes(P_F32);
    if ((e = mg->links.ensure(lbytes)) != hipSuccess || (e = mg->clover.ensure(cbytes)) != hipSuccess)
        return hip_fail(e, "gauge copy");
    if ((rc = hc(hipMemcpyAsync(mg->links.ptr, Gc->links, lbytes, hipMemcpyDeviceToDevice, st), "copy")) ||
        (rc = hc(hipMemcpyAsync(mg->clover.ptr, Gc->clover, cbytes, hipMemcpyDeviceToDevice, st), "copy")))
        return rc;
    mg->gauge.links = mg->links.ptr;
    mg->gauge.clover = mg->clover.ptr;
    mg->gauge.link_prec = P_F32;
    mg->gauge.clover_prec = P_F32;
    mg->gauge.eo = nullptr;
    const GaugeDev* G = &mg->gauge;
    if ((e = mg->P.ensure((size_t)nv * mg->field)) != hipSuccess) return hip_fail(e, "basis P");
    if ((e = mg->Dc.ensure((size_t)mg->nc * 9 * mg->n2 * mg->n2 * sizeof(float2))) != hipSuccess)
        return hip_fail(e, "coarse stencil");
    // fine workspace: the vectors, their next iterate, and the stencil-term chunk; all 2 N_v
    // columns of a term at once when the device has room (each restriction then reads P once
    // per term), else 16 at a time
    const size_t vbytes = (size_t)nv * mg->field;
    int chunk = std::min(mg->n2, 16);
    {
        size_t free_b = 0, total_b = 0;
        const size_t coarse_ws = (2 + coarse_work_vectors(mg.get(), params->coarse_restart)) * (size_t)nv *
                                 (size_t)(mg->nc * mg->n2) * sizeof(float2);
        const size_t need = 2 * vbytes + (size_t)mg->n2 * mg->field + coarse_ws + (size_t(4) << 30);
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && need <= free_b) chunk = mg->n2;
    }
    if ((e = mg->fine.ensure(2 * vbytes + (size_t)chunk * mg->field)) != hipSuccess) return hip_fail(e, "setup workspace");
    char* vcur = static_cast<char*>(mg->fine.ptr);
    char* vnext = vcur + vbytes;
    char* W = vnext + vbytes;
    if ((e = ds->stats.ensure(256)) != hipSuccess) return hip_fail(e, "stats");
    unsigned* flag = (unsigned*)ds->stats.ptr + 2;
    if ((rc = hc(hipMemsetAsync(flag, 0, sizeof(unsigned), st), "flag"))) return rc;
    if ((rc = hc(launch_spinor_import(mg->g, wrap_internal(vcur, mg->g, nv, P_F32), v0, flag, st), "import"))) return rc;
    unsigned bad = 0;
    if ((rc = hc(hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, st), "copy"))) return rc;
    if ((rc = hc(hipStreamSynchronize(st), "setup"))) return rc;
    if (bad) return fail(TM_ERR_NONFINITE, "non-finite starting vector");
    double mus[kMaxSys];
    for (int k = 0; k < kMaxSys; ++k) mus[k] = mg->mu0;
    for (int it = 1; it <= params->setup_iters; ++it) {
        const SpinorBuf vb = wrap_internal(vcur, mg->g, nv, P_F32), nb = wrap_internal(vnext, mg->g, nv, P_F32);
        if (it == 1)
            rc = run_sap(mg->g, *G, vb, nb, mus, nv, params->setup_cycles, params->mr_iters, true, 0, st);
        else
            rc = mg_apply(mg.get(), ds, vb, nb, mus, nv, st);
        if (rc) return rc;
        std::swap(vcur, vnext);
        if ((rc = orthonormalize_fields(mg.get(), reinterpret_cast<float2*>(vcur), nv, st))) return rc;
        if ((rc = build_coarse(mg.get(), *G, vcur, W, chunk, st))) return rc;
        if (verbose()) {
            (void)hipStreamSynchronize(st);
            std::fprintf(stderr, "[tm] two-level setup iteration %d of %d done at %.2f s\n", it, params->setup_iters,
                         std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
            std::fflush(stderr);
        }
    }
    if (params->setup_iters == 0 && (rc = build_coarse(mg.get(), *G, vcur, W, chunk, st))) return rc;
    if ((rc = hc(hipStreamSynchronize(st), "setup"))) return rc;
    // the setup's workspaces (test vectors, stencil terms, the coarse basis for n_vec systems)
    // are not needed by the solves
    mg->fine.release();
    mg->coarse.release();
    mg->applications = 0;
    mg->coarse_iters = 0;
    mg->t_coarse = 0;
    mg->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = mg.release();
    return TM_OK;
}

int tm_mg_destroy(tm_mg* mg) {
    delete mg;
    return TM_OK;
}

int tm_mg_get_info(const tm_mg* mg, tm_mg_info* info) {
    if (!mg || !info) return fail(TM_ERR_ARG, "null pointer");
    std::memset(info, 0, sizeof *info);
    for (int a = 0; a < 4; ++a) info->cdims[a] = mg->g.nb[a];
    info->n_vec = mg->p.n_vec;
    info->t_setup = mg->t_setup;
    info->applications = mg->applications;
    info->coarse_iters = mg->coarse_iters;
    info->t_coarse = mg->t_coarse;
    return TM_OK;
}

int tm_mg_export(tm_mg* mg, void* P, void* Dc, const tm_opts* opts) {
    int rc;
    if (!mg) return fail(TM_ERR_ARG, "mg is NULL");
    if ((rc = check_opts(opts)) || (rc = check_device(mg))) return rc;
    hipStream_t st = (hipStream_t)opts->stream;
    if (P && (rc = hc(launch_spinor_export(mg->g, wrap_internal(mg->P.ptr, mg->g, mg->p.n_vec, P_F32), P, st), "export")))
        return rc;
    if (Dc && (rc = hc(launch_mg_stencil_export(mg->nc, mg->p.n_vec, (const float2*)mg->Dc.ptr, Dc, st), "export")))
        return rc;
    return TM_OK;
}

int tm_mg_restrict(tm_mg* mg, int nsys, const void* r, void* c, const tm_opts* opts) {
    int rc;
    if (!mg || !r || !c) return fail(TM_ERR_ARG, "null pointer");
    if ((rc = check_opts(opts)) || (rc = check_device(mg))) return rc;
    if (nsys < 1 || nsys > kMaxSys) return fail(TM_ERR_ARG, "nsys = %d outside 1..%d", nsys, kMaxSys);
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    hipStream_t st = (hipStream_t)opts->stream;
    const long long n = mg->nc * mg->n2;
    hipError_t e;
    if ((e = ds->io.ensure((size_t)nsys * mg->field + (size_t)nsys * n * sizeof(float2))) != hipSuccess)
        return hip_fail(e, "workspace");
    if ((e = ds->stats.ensure(256)) != hipSuccess) return hip_fail(e, "stats");
    float2* cv = reinterpret_cast<float2*>(static_cast<char*>(ds->io.ptr) + (size_t)nsys * mg->field);
    if ((rc = hc(launch_spinor_import(mg->g, wrap_internal(ds->io.ptr, mg->g, nsys, P_F32), r, (unsigned*)ds->stats.ptr + 2,
                                      st), "import")))
        return rc;
    if ((rc = hc(launch_mg_restrict(margs(mg), ds->io.ptr, mg->field, nsys, cv, 0, (size_t)n, (size_t)mg->n2, st),
                 "restriction")))
        return rc;
    return hc(launch_mg_coarse_export(cv, c, (long long)nsys * n, st), "export");
}

int tm_mg_prolong(tm_mg* mg, int nsys, const void* c, void* e_out, const tm_opts* opts) {
    int rc;
    if (!mg || !c || !e_out) return fail(TM_ERR_ARG, "null pointer");
    if ((rc = check_opts(opts)) || (rc = check_device(mg))) return rc;
    if (nsys < 1 || nsys > kMaxSys) return fail(TM_ERR_ARG, "nsys = %d outside 1..%d", nsys, kMaxSys);
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    hipStream_t st = (hipStream_t)opts->stream;
    const long long n = mg->nc * mg->n2;
    hipError_t e;
    if ((e = ds->io.ensure((size_t)nsys * mg->field + (size_t)nsys * n * sizeof(float2))) != hipSuccess)
        return hip_fail(e, "workspace");
    if ((e = ds->stats.ensure(256)) != hipSuccess) return hip_fail(e, "stats");
    float2* cv = reinterpret_cast<float2*>(static_cast<char*>(ds->io.ptr) + (size_t)nsys * mg->field);
    if ((rc = hc(launch_mg_coarse_import(c, cv, (long long)nsys * n, (unsigned*)ds->stats.ptr + 2, st), "import")))
        return rc;
    if ((rc = hc(launch_mg_prolong(margs(mg), cv, nsys, ds->io.ptr, mg->field, st), "prolongation"))) return rc;
    return hc(launch_spinor_export(mg->g, wrap_internal(ds->io.ptr, mg->g, nsys, P_F32), e_out, st), "export");
}

int tm_mg_coarse_apply(tm_mg* mg, int nsys, const double* mu_c, const void* x, void* y, const tm_opts* opts) {
    int rc;
    if (!mg || !mu_c || !x || !y) return fail(TM_ERR_ARG, "null pointer");
    if ((rc = check_opts(opts)) || (rc = check_device(mg))) return rc;
    if (nsys < 1 || nsys > kMaxSys) return fail(TM_ERR_ARG, "nsys = %d outside 1..%d", nsys, kMaxSys);
    for (int k = 0; k < nsys; ++k)
        if (!std::isfinite(mu_c[k])) return fail(TM_ERR_ARG, "non-finite mu_c[%d]", k);
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    hipStream_t st = (hipStream_t)opts->stream;
    const long long n = mg->nc * mg->n2;
    hipError_t e;
    if ((e = ds->io.ensure(2 * (size_t)nsys * n * sizeof(float2) + 256 * sizeof(double))) != hipSuccess)
        return hip_fail(e, "workspace");
    if ((e = ds->stats.ensure(256)) != hipSuccess) return hip_fail(e, "stats");
    float2* xv = static_cast<float2*>(ds->io.ptr);
    float2* yv = xv + (size_t)nsys * n;
    double* mud = reinterpret_cast<double*>(yv + (size_t)nsys * n);
    if ((rc = hc(hipMemcpyAsync(mud, mu_c, nsys * sizeof(double), hipMemcpyHostToDevice, st), "copy"))) return rc;
    if ((rc = hc(launch_mg_coarse_import(x, xv, (long long)nsys * n, (unsigned*)ds->stats.ptr + 2, st), "import")))
        return rc;
    if ((rc = hc(launch_mg_coarse_apply(mg->g, mg->p.n_vec, (const float2*)mg->Dc.ptr, mud, xv, yv, nsys, st),
                 "coarse operator")))
        return rc;
    if ((rc = hc(launch_mg_coarse_export(yv, y, (long long)nsys * n, st), "export"))) return rc;
    return hc(hipStreamSynchronize(st), "coarse operator");
}

int tm_mg_coarse_solve(tm_mg* mg, int nsys, const double* mu_c, const void* b, void* x, double tol, int restart,
                       int max_restarts, int* iters, const tm_opts* opts) {
    int rc;
    if (!mg || !mu_c || !b || !x) return fail(TM_ERR_ARG, "null pointer");
    if ((rc = check_opts(opts)) || (rc = check_device(mg))) return rc;
    if (nsys < 1 || nsys > kMaxSys) return fail(TM_ERR_ARG, "nsys = %d outside 1..%d", nsys, kMaxSys);
    if (restart < 1 || restart > 128 || max_restarts < 1) return fail(TM_ERR_ARG, "restart 1..128, max_restarts >= 1");
    if (!(tol >= 0) || !std::isfinite(tol)) return fail(TM_ERR_ARG, "bad tol");
    for (int k = 0; k < nsys; ++k)
        if (!std::isfinite(mu_c[k])) return fail(TM_ERR_ARG, "non-finite mu_c[%d]", k);
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    hipStream_t st = (hipStream_t)opts->stream;
    const long long n = mg->nc * mg->n2;
    hipError_t e;
    if ((e = ds->io.ensure(2 * (size_t)nsys * n * sizeof(float2))) != hipSuccess) return hip_fail(e, "workspace");
    if ((e = ds->stats.ensure(256)) != hipSuccess) return hip_fail(e, "stats");
    float2* bv = static_cast<float2*>(ds->io.ptr);
    float2* xv = bv + (size_t)nsys * n;
    if ((rc = hc(launch_mg_coarse_import(b, bv, (long long)nsys * n, (unsigned*)ds->stats.ptr + 2, st), "import")))
        return rc;
    if ((rc = mg_coarse_gmres(mg, nsys, mu_c, bv, xv, tol, restart, max_restarts, iters, st))) return rc;
    if ((rc = hc(launch_mg_coarse_export(xv, x, (long long)nsys * n, st), "export"))) return rc;
    return hc(hipStreamSynchronize(st), "coarse solve");
}

int tm_mg_precond(const tm_geom* geom, tm_mg* mg, const void* r, void* z, const tm_opts* opts) {
    int rc;
    if (!mg || !r || !z) return fail(TM_ERR_ARG, "null pointer");
    if ((rc = check_geom(geom)) || (rc = check_opts(opts)) || (rc = check_storage(opts)) || (rc = mg_matches(mg, geom)))
        return rc;
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    hipStream_t st = (hipStream_t)opts->stream;
    const int ns = geom->nsys;
    hipError_t e;
    if ((e = ds->io.ensure(2 * (size_t)ns * mg->field)) != hipSuccess) return hip_fail(e, "workspace");
    if ((e = ds->stats.ensure(256)) != hipSuccess) return hip_fail(e, "stats");
    const SpinorBuf rb = wrap_internal(ds->io.ptr, mg->g, ns, P_F32);
    const SpinorBuf zb = wrap_internal(static_cast<char*>(ds->io.ptr) + (size_t)ns * mg->field, mg->g, ns, P_F32);
    if ((rc = hc(launch_spinor_import(mg->g, rb, r, (unsigned*)ds->stats.ptr + 2, st), "import"))) return rc;
    double mu[kMaxSys];
    fill_mu(geom, mu);
    if ((rc = mg_apply(mg, ds, rb, zb, mu, ns, st))) return rc;
    if ((rc = hc(launch_spinor_export(mg->g, zb, z, st), "export"))) return rc;
    return hc(hipStreamSynchronize(st), "two-level preconditioner");
}

}  // extern "C"
