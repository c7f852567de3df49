// CG on the squared even-odd reduced system: the plain FP64 baseline of the
// paper's comparison (section 3: CG on Dhat^+ Dhat x = Dhat^+ b', eq.
// (oereduced) for Dhat = D_ee - D_eo D_oo^-1 D_oe).
//
// Run in the least-squares form: r = bhat - Dhat x_e is the reduced residual
// and s = Dhat^+ r the residual of the normal equations.  With
// x_o = D_oo^-1 (b_o - D_oe x_e) the odd rows of b - D x vanish and the even
// rows equal r, so ||r|| <= tol ||b|| is the stopping test.  r is updated
// recursively; the returned status rests on the true residual b - D x
// recomputed with the full operator, and CG restarts from it when rounding
// left it above tol.  All systems of a group advance together; a converged
// system takes zero steps from then on.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/tm.h"
#include "tm_api_internal.h"
#include "tm_blas.h"

namespace tmsap {

namespace {

int hchk(hipError_t e, const char* where) { return e == hipSuccess ? TM_OK : hip_fail(e, where); }

struct CgCtx {
    Geo g;
    const GaugeDev* G;
    hipStream_t st;
    int ns;
    double mu[kMaxSys];
    const void* inv[kMaxEoMu];
    unsigned char sel[kMaxSys];
    long long half;
    double* partials;
};

ParityArgs base_args(const CgCtx& c, int p) {
    ParityArgs a;
    std::memset(&a, 0, sizeof a);
    a.g = c.g;
    a.links = c.G->links;
    a.clover = c.G->clover;
    for (int k = 0; k < kMaxEoMu; ++k) a.inv[k] = c.inv[k];
    for (int k = 0; k < kMaxSys; ++k) {
        a.sel[k] = c.sel[k];
        a.mu[k] = c.mu[k];
    }
    a.p = p;
    a.hop_sign = 1.0;
    a.add_sign = 1.0;
    a.mu_sign = 1.0;
    a.nsys = c.ns;
    return a;
}

// out = Dhat in (adj: Dhat^+ in = Gamma5 Dhat(-mu) Gamma5 in); t: odd-parity scratch
int dhat(const CgCtx& c, const double* in, double* t, double* out, bool adj) {
    ParityArgs a = base_args(c, 1);  // t_o = D_oo^-1 H_oe in
    a.in_hop = in;
    a.do_inv = 1;
    a.g5_hop = adj;
    a.mu_sign = adj ? -1.0 : 1.0;
    a.out = t;
    int rc;
    if ((rc = hchk(launch_parity_op(a, c.st), "reduced operator"))) return rc;
    ParityArgs b = base_args(c, 0);  // out_e = D_ee in - H_eo t_o
    b.in_diag = in;
    b.g5_diag = adj;
    b.in_hop = t;
    b.hop_sign = -1.0;
    b.g5_out = adj;
    b.mu_sign = adj ? -1.0 : 1.0;
    b.out = out;
    return hchk(launch_parity_op(b, c.st), "reduced operator");
}

VecRef compact_ref(double* p, long long half) {
    VecRef r;
    r.data = p;
    r.scale = nullptr;
    r.sys_stride = (size_t)6 * half * 32;
    return r;
}

// out[sys] = ||v_sys||^2
int norm2(const CgCtx& c, double* v, double* out) {
    const VecRef r = compact_ref(v, c.half);
    return hchk(blas_norm2(P_F64, r, c.partials, out, c.ns, c.half, c.st), "norm");
}

}  // namespace

}  // namespace tmsap

using namespace tmsap;

extern "C" {

int tm_cg_solve(const tm_geom* geom, const void* U, const void* b, void* x, double kappa, double c_sw, double tol,
                int max_iters, const tm_opts* opts, tm_solve_report* report) {
    const auto t_start = std::chrono::steady_clock::now();
    int rc;
    if ((rc = check_geom(geom)) || (rc = check_opts(opts))) return rc;
    if (!U || !b || !x) return fail(TM_ERR_ARG, "null pointer");
    if (b == x) return fail(TM_ERR_ARG, "b and x alias");
    if (opts->io != TM_IO_CANONICAL) return fail(TM_ERR_ARG, "tm_cg_solve takes canonical buffers");
    if (opts->storage != TM_F64) return fail(TM_ERR_PREC, "the CG baseline runs in FP64 (storage TM_F64)");
    if (!(tol > 0) || !(kappa > 0) || !std::isfinite(c_sw) || max_iters < 1)
        return fail(TM_ERR_ARG, "bad tol, kappa, c_sw or max_iters");
    for (int a = 0; a < 4; ++a)
        if (geom->dims[a] % 2 != 0)
            return fail(TM_ERR_DIMS, "even-odd reduction needs even dims (dims[%d] = %d)", a, geom->dims[a]);
    int tile[4];
    if ((rc = choose_tile(geom, opts->layout_block, tile))) return rc;
    if (tile[3] % 2 != 0) return fail(TM_ERR_BLOCKS, "layout tile needs an even x-extent");
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    hipStream_t st = (hipStream_t)opts->stream;
    const Geo g = make_geo(geom, tile);
    const long long half = g.V / 2;
    const GaugeDev* G;
    if ((rc = get_gauge(ds, g, U, kappa, c_sw, P_F64, opts->gauge_tag, st, &G))) return rc;

    // per system: 8 compact FP64 fields + 3 full FP64 fields for the closing residual
    const size_t cfield = (size_t)6 * half * 32, ffield = internal_bytes(g, 1, P_F64);
    const int group = fit_group(ds, geom->nsys, 0, 8 * cfield + 3 * ffield, 0);

    tm_solve_report rep;
    std::memset(&rep, 0, sizeof rep);
    int all_conv = 1;
    const size_t canon_sys = (size_t)g.V * 12 * 2 * sizeof(double);
    std::vector<double> host(8 * kMaxSys);
    for (int g0 = 0; g0 < geom->nsys; g0 += group) {
        const int ns = std::min(group, geom->nsys - g0);
        CgCtx c;
        c.g = g;
        c.G = G;
        c.st = st;
        c.ns = ns;
        c.half = half;
        for (int k = 0; k < kMaxSys; ++k) c.mu[k] = k < ns ? geom->mu[g0 + k] : 0.0;
        unsigned long long adj = 0;  // the kernels take the adjoint from the sign of the effective mu
        for (int k = 0; k < kMaxEoMu; ++k) c.inv[k] = nullptr;
        double muo[kMaxSys];  // the twist on the odd sites, whose inverses D_oo^-1 uses
        for (int k = 0; k < ns; ++k) muo[k] = c.mu[k] + g.mu_shift[1];
        if ((rc = prepare_site_inverses(g, *G, muo, ns, 1, st, c.inv, c.sel, &adj))) return rc;

        hipError_t h = ds->solver.ensure(8 * cfield * ns);
        if (h != hipSuccess) return hip_fail(h, "CG workspace");
        double* base = (double*)ds->solver.ptr;
        const size_t fd = cfield * ns / sizeof(double);
        double *be = base, *bo = base + fd, *xe = base + 2 * fd, *r = base + 3 * fd, *s = base + 4 * fd,
               *p = base + 5 * fd, *q = base + 6 * fd, *t = base + 7 * fd;
        // scalars: gamma, qq, rr, alpha, -alpha, beta, one, zero / -one, gnew, b-norms
        const int nblk = blas_blocks(half);
        const int nblk_full = blas_blocks(g.V);
        if ((h = ds->red.ensure((16 * kMaxSys + 2 * (size_t)kMaxSys * std::max(nblk, nblk_full) + 64) *
                                sizeof(double))) != hipSuccess)
            return hip_fail(h, "CG scalars");
        double* sc = (double*)ds->red.ptr;
        double *gam = sc, *qq = sc + kMaxSys, *rr = sc + 2 * kMaxSys, *alpha = sc + 3 * kMaxSys,
               *nalpha = sc + 4 * kMaxSys, *beta = sc + 5 * kMaxSys, *one = sc + 6 * kMaxSys,
               *zero = sc + 7 * kMaxSys, *mone = sc + 8 * kMaxSys, *gnew = sc + 9 * kMaxSys,
               *bn1 = sc + 10 * kMaxSys, *bn2 = sc + 11 * kMaxSys;
        c.partials = sc + 16 * kMaxSys;
        for (int k = 0; k < kMaxSys; ++k) {
            host[k] = 1.0;
            host[kMaxSys + k] = 0.0;
            host[2 * kMaxSys + k] = -1.0;
        }
        if ((rc = hchk(hipMemcpyAsync(one, host.data(), 3 * kMaxSys * sizeof(double), hipMemcpyHostToDevice, st),
                       "copy")))
            return rc;
        if ((h = ds->stats.ensure(256)) != hipSuccess) return hip_fail(h, "stats");
        unsigned* flag = (unsigned*)ds->stats.ptr + 2;
        if ((rc = hchk(hipMemsetAsync(flag, 0, sizeof(unsigned), st), "memset"))) return rc;
        const char* bcan = (const char*)b + g0 * canon_sys;
        char* xcan = (char*)x + g0 * canon_sys;
        if ((rc = hchk(launch_parity_import(g, ns, bcan, be, bo, flag, st), "import b"))) return rc;
        if ((rc = hchk(launch_parity_import(g, ns, xcan, xe, t, flag, st), "import x"))) return rc;
        // Each pass runs CG from the current x_e on the recomputed reduced residual, then forms x_o and
        // the true residual b - D x with the full operator.  A system is converged when that true
        // residual is <= tol ||b||; one whose recursively updated residual met tol while the true one
        // did not (rounding drift) goes through another pass, at most 3 more, within max_iters steps.
        std::vector<double> bnorm(ns);
        std::vector<int> iters(ns, 0);
        unsigned long long met = 0;  // systems whose true residual is <= tol
        const unsigned long long all = ns == 64 ? ~0ull : ((1ull << ns) - 1);
        int it = 0;
        for (int pass = 0;; ++pass) {
            // ||b||^2 (the closing residual of a pass reuses these scalars)
            if ((rc = norm2(c, be, bn1)) || (rc = norm2(c, bo, bn2))) return rc;
            // r = bhat - Dhat x_e with bhat = b_e - H_eo D_oo^-1 b_o
            ParityArgs a0 = base_args(c, 1);
            a0.in_add = bo;
            a0.do_inv = 1;
            a0.out = t;
            if ((rc = hchk(launch_parity_op(a0, st), "reduced rhs"))) return rc;
            ParityArgs a1 = base_args(c, 0);
            a1.in_add = be;
            a1.in_hop = t;
            a1.hop_sign = -1.0;
            a1.out = r;
            if ((rc = hchk(launch_parity_op(a1, st), "reduced rhs"))) return rc;
            if ((rc = dhat(c, xe, t, q, false))) return rc;
            if ((rc = hchk(launch_axpby(q, mone, r, one, ns, (long long)fd / ns, st), "axpby"))) return rc;
            // s = Dhat^+ r, p = s, gamma = ||s||^2
            if ((rc = dhat(c, r, t, s, true))) return rc;
            if ((rc = hchk(launch_axpby(s, one, p, zero, ns, (long long)fd / ns, st), "axpby"))) return rc;
            if ((rc = norm2(c, s, gam))) return rc;
            if ((rc = norm2(c, r, rr))) return rc;
            if ((rc = hchk(hipMemcpyAsync(host.data(), bn1, 2 * kMaxSys * sizeof(double), hipMemcpyDeviceToHost, st),
                           "copy")))
                return rc;
            if ((rc = hchk(hipMemcpyAsync(host.data() + 2 * kMaxSys, rr, ns * sizeof(double), hipMemcpyDeviceToHost, st),
                           "copy")))
                return rc;
            unsigned hflag = 0;
            if ((rc = hchk(hipMemcpyAsync(&hflag, flag, sizeof hflag, hipMemcpyDeviceToHost, st), "copy"))) return rc;
            if ((rc = hchk(hipStreamSynchronize(st), "CG setup"))) return rc;
            if (hflag) return fail(TM_ERR_NONFINITE, "b or x holds NaN or Inf");
            unsigned long long frozen = met;
            for (int k = 0; k < ns; ++k) {
                bnorm[k] = std::sqrt(host[k] + host[kMaxSys + k]);
                const double rk = std::sqrt(std::max(0.0, host[2 * kMaxSys + k]));
                if (!std::isfinite(rk)) return fail(TM_ERR_NONFINITE, "non-finite CG residual");
                if (rk <= tol * bnorm[k]) frozen |= 1ull << k;
            }
            while (frozen != all && it < max_iters) {
                if ((rc = dhat(c, p, t, q, false))) return rc;
                if ((rc = norm2(c, q, qq))) return rc;
                if ((rc = hchk(launch_cg_scalars(0, ns, frozen, gam, qq, alpha, nalpha, st), "scalars"))) return rc;
                if ((rc = hchk(launch_axpby(p, alpha, xe, one, ns, (long long)fd / ns, st), "axpby"))) return rc;
                if ((rc = hchk(launch_axpby(q, nalpha, r, one, ns, (long long)fd / ns, st), "axpby"))) return rc;
                if ((rc = norm2(c, r, rr))) return rc;
                if ((rc = hchk(hipMemcpyAsync(host.data(), rr, ns * sizeof(double), hipMemcpyDeviceToHost, st), "copy")))
                    return rc;
                if ((rc = dhat(c, r, t, s, true))) return rc;
                if ((rc = norm2(c, s, gnew))) return rc;
                if ((rc = hchk(launch_cg_scalars(1, ns, frozen, gam, gnew, beta, nullptr, st), "scalars"))) return rc;
                if ((rc = hchk(launch_axpby(s, one, p, beta, ns, (long long)fd / ns, st), "axpby"))) return rc;
                if ((rc = hchk(hipStreamSynchronize(st), "CG step"))) return rc;
                ++it;
                for (int k = 0; k < ns; ++k) {
                    if ((frozen >> k) & 1ull) continue;
                    ++iters[k];
                    const double rk = std::sqrt(std::max(0.0, host[k]));
                    if (!std::isfinite(host[k])) return fail(TM_ERR_NONFINITE, "non-finite CG residual");
                    if (rk <= tol * bnorm[k]) frozen |= 1ull << k;
                }
            }
            // x_o = D_oo^-1 (b_o - H_oe x_e), then back to the canonical layout
            ParityArgs a2 = base_args(c, 1);
            a2.in_add = bo;
            a2.in_hop = xe;
            a2.hop_sign = -1.0;
            a2.do_inv = 1;
            a2.out = t;
            if ((rc = hchk(launch_parity_op(a2, st), "odd sites"))) return rc;
            if ((rc = hchk(launch_parity_export(g, ns, xe, t, xcan, st), "export x"))) return rc;

            // true residual b - D x with the full operator
            if ((h = ds->io.ensure(3 * ffield * ns)) != hipSuccess) return hip_fail(h, "residual workspace");
            SpinorBuf fb = wrap_internal(ds->io.ptr, g, ns, P_F64);
            SpinorBuf fx = wrap_internal((char*)ds->io.ptr + ffield * ns, g, ns, P_F64);
            SpinorBuf fr = wrap_internal((char*)ds->io.ptr + 2 * ffield * ns, g, ns, P_F64);
            if ((rc = hchk(launch_spinor_import(g, fb, bcan, flag, st), "import"))) return rc;
            if ((rc = hchk(launch_spinor_import(g, fx, xcan, flag, st), "import"))) return rc;
            if ((rc = run_dirac(g, *G, fx, fr, c.mu, ns, P_F64, st))) return rc;
            if ((rc = hchk(blas_residual(P_F64, vec_ref(fb, g.V), vec_ref(fr, g.V), vec_ref(fr, g.V), c.partials, bn1, ns,
                                         g.V, st, P_F64),
                           "residual")))
                return rc;
            if ((rc = hchk(hipMemcpyAsync(host.data(), bn1, 2 * ns * sizeof(double), hipMemcpyDeviceToHost, st), "copy")))
                return rc;
            if ((rc = hchk(hipStreamSynchronize(st), "residual"))) return rc;
            met = 0;
            for (int k = 0; k < ns; ++k) {
                const double rel = host[2 * k + 1] > 0 ? std::sqrt(host[2 * k] / host[2 * k + 1]) : 0.0;
                rep.true_rel_res[g0 + k] = rel;
                if (rel <= tol) met |= 1ull << k;
            }
            if (met == all || it >= max_iters || pass >= 3) break;
        }
        for (int k = 0; k < ns; ++k) {
            const bool ok = ((met >> k) & 1ull) != 0;
            rep.converged += ok;
            all_conv &= ok;
            rep.iters = std::max(rep.iters, iters[k]);
        }
        rep.group = ns;
    }
    rep.t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (report) *report = rep;
    return all_conv ? TM_OK : TM_NOT_CONVERGED;
}

}  // extern "C"
