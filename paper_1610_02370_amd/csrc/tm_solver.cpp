// Flexible GMRES right-preconditioned by SAP (section 2.5), the mixed-
// precision defect-correction form (section 3.1: an FP64 residual loop around
// FP32 FGMRES solves to a relative 1e-6).
//
// All systems of a group advance together; each keeps its own Hessenberg
// matrix, Givens rotations and Krylov dimension.  A system whose residual
// estimate reaches the tolerance is frozen: its next basis vectors are zero,
// so batched kernels carry it at no effect.  Orthogonalisation is classical
// Gram-Schmidt with delayed reorthogonalisation in two sweeps over the stored
// directions per step, the orthonormal basis kept implicit through a small
// triangular factor; the host reads one Hessenberg column per step (the
// previous one finished, the current one provisional) and solves the small
// least-squares problems.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tm.h"
#include "tm_api_internal.h"
#include "tm_blas.h"

namespace tmsap {

namespace {

typedef std::complex<double> zc;

// TM_VERBOSE=1: one progress line per Arnoldi step and per outer
// defect-correction step on stderr.
bool verbose() {
    static int v = -1;
    if (v < 0) {
        const char* e = std::getenv("TM_VERBOSE");
        v = (e && e[0] && e[0] != '0') ? 1 : 0;
    }
    return v == 1;
}

struct Pinned {
    double* p = nullptr;
    size_t n = 0;
    ~Pinned() {
        if (p) (void)hipHostFree(p);
    }
    hipError_t ensure(size_t count) {
        if (count <= n) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipHostMalloc((void**)&p, count * sizeof(double), hipHostMallocDefault);
        if (e == hipSuccess) n = count;
        return e;
    }
};

// Device scratch of one solve (carved from the device's reduction buffer).
struct Scratch {
    double* inv;       // [nsys]
    double* ones;      // [nsys]
    double* y;         // [nsys][kMaxVec][2]
    double* res;       // [nsys][2]
    double* dots;      // [nsys][4 kMaxVec] Gram-Schmidt dots
    double* coef;      // [nsys][4 kMaxVec] update coefficients
    double* rep;       // [nsys][4 + 4 kMaxVec] beta, h, s, V^H u, V^H w
    double* nrm2;      // [nsys] norm of the update sweep's output
    double* tri;       // [nsys][kMaxVec][kMaxVec] complex: U = V T
    double* partials;  // [nsys * 2 * kMaxVec][blocks]
};

struct Ctx {
    DeviceState* ds;
    hipStream_t st;
    Geo g;
    int nsys;
    double mu[kMaxSys];
    int n_cycles, mr_iters;
    int sys_tile;  // SAP systems per workgroup (0 = all)
    bool eo;       // even-odd preconditioned SAP block solves
    const GaugeDev* op;  // operator for w = D z and residuals
    Prec op_compute;
    const GaugeDev* sap;  // smoother gauge
    tm_mg* mg = nullptr;  // two-level preconditioner (else SAP)
    Prec vp;              // Krylov vectors
    Prec sp;              // smoother storage (preconditioned vectors z)
    Scratch sc;
    Pinned host;      // pinned host memory: [stage | inv | y], one region per transfer purpose
    double* hstage = nullptr;  // device -> host Hessenberg columns and norms
    double* hinv = nullptr;    // host -> device 1/beta and 1/||w|| factors
    double* hy = nullptr;      // host -> device least-squares solutions
    hipEvent_t ev[2];
    double t_sap = 0;
    long long sap_cycles = 0;
    long long sap_sys_cycles = 0;
};

int hcheck(hipError_t e, const char* where) { return e == hipSuccess ? TM_OK : hip_fail(e, where); }

// Krylov storage: the m+1 once-projected directions u_i (at vp; the orthonormal basis is
// V = U T^-1, T kept by the Gram-Schmidt kernels), Z (m at sp), w (vp), vS (sp, when sp != vp).
struct Krylov {
    int m;
    char* V;
    size_t vstride;
    char* Z;
    size_t zstride;
    SpinorBuf w;
    SpinorBuf vS;
    bool convert;

    SpinorBuf Vb(const Ctx& c, int i) const { return wrap_internal(V + i * vstride, c.g, c.nsys, c.vp); }
    SpinorBuf Zb(const Ctx& c, int i) const { return wrap_internal(Z + i * zstride, c.g, c.nsys, c.sp); }
};

size_t krylov_bytes(const Geo& g, int nsys, int m, Prec vp, Prec sp) {
    size_t v = internal_bytes(g, nsys, vp), z = internal_bytes(g, nsys, sp);
    return (size_t)(m + 2) * v + (size_t)m * z + (sp != vp ? z : 0);
}

Krylov carve_krylov(char*& p, const Geo& g, int nsys, int m, Prec vp, Prec sp) {
    Krylov k;
    k.m = m;
    k.vstride = internal_bytes(g, nsys, vp);
    k.zstride = internal_bytes(g, nsys, sp);
    k.V = p;
    p += (size_t)(m + 1) * k.vstride;
    k.Z = p;
    p += (size_t)m * k.zstride;
    k.w = wrap_internal(p, g, nsys, vp);
    p += k.vstride;
    k.convert = sp != vp;
    if (k.convert) {
        k.vS = wrap_internal(p, g, nsys, sp);
        p += k.zstride;
    }
    return k;
}

// r = rhs - D x; host gets ||r||^2 and ||rhs||^2.  When x is zero the residual is rhs
// itself: r is not written, only the norm of rhs is taken.  With rout, r holds D x and the
// residual goes to rout instead (at rout's precision: FP64 rounded once to FP32).
int residual(Ctx& c, const SpinorBuf& rhs, const SpinorBuf& x, bool x_zero, const SpinorBuf& r, double* rn2,
             double* bn2, const SpinorBuf* rout = nullptr) {
    const long long V = c.g.V;
    int rc;
    if (x_zero) {
        if ((rc = hcheck(blas_norm2(c.vp, vec_ref(rhs, V), c.sc.partials, c.sc.res, c.nsys, V, c.st), "norm")))
            return rc;
        if ((rc = hcheck(hipMemcpyAsync(c.hstage, c.sc.res, c.nsys * sizeof(double), hipMemcpyDeviceToHost, c.st),
                         "copy")))
            return rc;
        if ((rc = hcheck(hipStreamSynchronize(c.st), "residual"))) return rc;
        for (int k = 0; k < c.nsys; ++k) rn2[k] = bn2[k] = c.hstage[k];
        return TM_OK;
    }
    if ((rc = run_dirac(c.g, *c.op, x, r, c.mu, c.nsys, c.op_compute, c.st))) return rc;
    const SpinorBuf& ro = rout ? *rout : r;
    if ((rc = hcheck(blas_residual(c.vp, vec_ref(rhs, V), vec_ref(r, V), vec_ref(ro, V), c.sc.partials, c.sc.res,
                                   c.nsys, V, c.st, ro.prec),
                     "residual")))
        return rc;
    if ((rc = hcheck(hipMemcpyAsync(c.hstage, c.sc.res, 2 * c.nsys * sizeof(double), hipMemcpyDeviceToHost, c.st),
                     "copy")))
        return rc;
    if ((rc = hcheck(hipStreamSynchronize(c.st), "residual"))) return rc;
    for (int k = 0; k < c.nsys; ++k) {
        rn2[k] = c.hstage[2 * k];
        bn2[k] = c.hstage[2 * k + 1];
        if (!std::isfinite(rn2[k])) return fail(TM_ERR_NONFINITE, "non-finite residual of system %d", k);
    }
    return TM_OK;
}

struct CoreResult {
    int iters[kMaxSys];
    double rel[kMaxSys];
    bool conv[kMaxSys];
    bool accumulated;  // the solution was added to x_acc (x left as it was)
};

// FGMRES(m) for D x = rhs, x in/out, all vectors at c.vp.  Stops per system k at
// ||rhs - D x|| <= tol[k] ||rhs|| (residual recomputed at every restart at the
// operator's precision) or when max_iters Arnoldi steps were taken.  Systems
// in the `skip` mask are frozen from the start and keep x as it is.  x_zero:
// x is taken as zero and its contents are not read.  With trust_estimate, a
// cycle in which every system met its tolerance by the least-squares residual
// estimate ends the solve without recomputing the residual (out.rel then holds
// the estimates): for inner solves whose caller computes the true residual
// next.  With x_acc (FP64, same systems), a solve from zero that ends that way
// in its first cycle adds its solution to *x_acc instead of writing x
// (out.accumulated; with x_acc_zero, *x_acc is taken as zero and overwritten).
int fgmres_core(Ctx& c, Krylov& K, const SpinorBuf& rhs, const SpinorBuf& x, bool x_zero, const double* tol,
                int max_iters, CoreResult& out, unsigned long long skip = 0, bool trust_estimate = false,
                const SpinorBuf* x_acc = nullptr, bool x_acc_zero = false) {
    const long long V = c.g.V;
    const int ns = c.nsys, m = K.m;
    int rc;
    std::vector<double> rn2(ns), bn2(ns), bnorm(ns);
    // per system: the Hessenberg columns as formed (Hraw) and after the Givens rotations (R), the
    // rotations, and the rotated right-hand side g
    std::vector<zc> Hraw((size_t)ns * (m + 1) * m), R((size_t)ns * (m + 1) * m), sn((size_t)ns * m),
        gv((size_t)ns * (m + 1)), gsave(ns);
    std::vector<double> cs((size_t)ns * m), sprev(ns);
    std::vector<int> kdim(ns);
    std::vector<char> frozen(ns);
    // rotate column j of system k by the rotations of columns < j, form the rotation of column j
    // and apply it to g (g_j, g_{j+1})
    auto commit = [&](int k, int j) {
        const zc* Hk = &Hraw[(size_t)k * (m + 1) * m];
        zc* Rk = &R[(size_t)k * (m + 1) * m];
        double* csk = &cs[(size_t)k * m];
        zc* snk = &sn[(size_t)k * m];
        zc* gk = &gv[(size_t)k * (m + 1)];
        for (int i = 0; i <= j + 1; ++i) Rk[i * m + j] = Hk[i * m + j];
        for (int i = 0; i < j; ++i) {
            const zc a = Rk[i * m + j], b2 = Rk[(i + 1) * m + j];
            Rk[i * m + j] = csk[i] * a + snk[i] * b2;
            Rk[(i + 1) * m + j] = -std::conj(snk[i]) * a + csk[i] * b2;
        }
        const zc a = Rk[j * m + j], b2 = Rk[(j + 1) * m + j];
        const double t = std::sqrt(std::norm(a) + std::norm(b2));
        if (std::abs(a) == 0.0) {
            csk[j] = 0.0;
            snk[j] = 1.0;
        } else {
            csk[j] = std::abs(a) / t;
            snk[j] = (a / std::abs(a)) * std::conj(b2) / t;
        }
        Rk[j * m + j] = csk[j] * a + snk[j] * b2;
        Rk[(j + 1) * m + j] = 0.0;
        gk[j + 1] = -std::conj(snk[j]) * gk[j];
        gk[j] = csk[j] * gk[j];
    };
    for (int k = 0; k < ns; ++k) out.iters[k] = 0;
    out.accumulated = false;
    SpinorBuf V0 = K.Vb(c, 0);
    if ((rc = residual(c, rhs, x, x_zero, V0, rn2.data(), bn2.data()))) return rc;
    bool r_in_rhs = x_zero;  // the residual is rhs itself until x changes
    for (int k = 0; k < ns; ++k) bnorm[k] = std::sqrt(bn2[k]);
    int steps = 0;
    // systems whose preconditioned direction vanished (a zero pivot in the first column of a
    // cycle: no progress possible) are not cycled again; they end unconverged
    unsigned long long stalled = 0;
    for (;;) {
        bool any = false;
        for (int k = 0; k < ns; ++k) {
            const double rel = bnorm[k] > 0 ? std::sqrt(rn2[k]) / bnorm[k] : 0.0;
            out.rel[k] = rel;
            out.conv[k] = rel <= tol[k] || ((skip >> k) & 1ull);
            frozen[k] = out.conv[k] || ((stalled >> k) & 1ull);
            any |= !frozen[k];
        }
        if (!any || steps >= max_iters) break;
        // v0 = r / beta
        for (int k = 0; k < ns; ++k) {
            const double beta = std::sqrt(rn2[k]);
            c.hinv[k] = frozen[k] ? 0.0 : 1.0 / beta;
            for (int i = 0; i <= m; ++i) gv[(size_t)k * (m + 1) + i] = 0;
            gv[(size_t)k * (m + 1)] = frozen[k] ? 0.0 : beta;
            kdim[k] = 0;
        }
        if ((rc = hcheck(hipMemcpyAsync(c.sc.inv, c.hinv, ns * sizeof(double), hipMemcpyHostToDevice, c.st), "copy")))
            return rc;
        if ((rc = hcheck(blas_scale(c.vp, c.vp, vec_ref(r_in_rhs ? rhs : V0, V), c.sc.inv, vec_ref(V0, V), ns, V,
                                    c.st),
                         "scale")))
            return rc;
        r_in_rhs = false;
        int jdone = 0;
        for (int j = 0; j < m && steps < max_iters; ++j) {
            // slot j: v_0 at the first step, afterwards the direction u_j of the previous step,
            // orthogonalised once; it becomes v_j in this step's update sweep
            const SpinorBuf uj = K.Vb(c, j);
            const SpinorBuf zj = K.Zb(c, j);
            SpinorBuf src = uj;
            if (K.convert) {
                if ((rc = hcheck(launch_spinor_convert(c.g, uj, K.vS, c.st), "convert"))) return rc;
                src = K.vS;
            }
            // z_j = SAP(u_j) from a zero guess; w = D z_j.  When the smoother and the operator
            // share the FP32 gauge copy and z_j is stored in FP32, the last half-sweep gives D z_j on
            // its own blocks (b minus the blocks' final residual), so the operator runs on the
            // other colour's blocks only.
            const bool w_from_sap = !c.mg && c.sap == c.op && c.op_compute == P_F32 && K.w.prec == P_F32 &&
                                    zj.prec == P_F32 &&
                                    sap_fills_w(c.g, src.prec, c.sap->link_prec, c.sap->clover_prec, c.eo);
            if ((rc = hcheck(hipEventRecord(c.ev[0], c.st), "event"))) return rc;
            if (c.mg)
                rc = mg_apply(c.mg, c.ds, src, zj, c.mu, ns, c.st);
            else
                rc = run_sap(c.g, *c.sap, src, zj, c.mu, ns, c.n_cycles, c.mr_iters, true, c.sys_tile, c.st, c.eo,
                             w_from_sap ? K.w.data : nullptr);
            if (rc) return rc;
            if ((rc = hcheck(hipEventRecord(c.ev[1], c.st), "event"))) return rc;
            c.sap_cycles += c.n_cycles;
            c.sap_sys_cycles += (long long)c.n_cycles * ns;
            if (w_from_sap)
                rc = run_dirac_colour(c.g, *c.op, zj, K.w, c.mu, ns, 0, c.st);
            else
                rc = run_dirac(c.g, *c.op, zj, K.w, c.mu, ns, c.op_compute, c.st);
            if (rc) return rc;
            // classical Gram-Schmidt with delayed reorthogonalisation: one sweep for the dots of the
            // stored directions u_0..u_{j-1} with u_j and w (and <u,u>, <u,w>, <w,w>), a small
            // kernel that takes them to the orthonormal basis V = U T^-1 and finishes v_j =
            // (u_j - V V^H u_j) / beta implicitly (column j of T), then one sweep that writes
            // u_{j+1} = s (w - V_j V_j^H w), projected once; its second projection is the first part
            // of the next step.  V itself is never stored.
            const VecRef basis = vec_ref(K.Vb(c, 0), V), wr = vec_ref(K.w, V), ur = vec_ref(uj, V);
            const SpinorBuf un = K.Vb(c, j + 1);
            unsigned long long off = 0;
            for (int k = 0; k < ns; ++k)
                if (frozen[k]) off |= 1ull << k;
            if ((rc = hcheck(blas_dgs_dots(c.vp, basis, K.vstride, j, ur, wr, c.sc.partials, c.sc.dots, ns, V, c.st),
                             "gs")))
                return rc;
            if ((rc = hcheck(blas_dgs_coef(c.sc.dots, j, ns, off, c.sc.coef, c.sc.rep, c.sc.tri, c.st), "gs")))
                return rc;
            if ((rc = hcheck(blas_dgs_update(c.vp, basis, K.vstride, j, ur, wr, vec_ref(un, V), c.sc.coef,
                                             c.sc.partials, c.sc.nrm2, ns, V, c.st),
                             "gs")))
                return rc;
            const size_t rstride = 4 + 4 * (size_t)blas_dgs_tri_stride();
            double* st_rep = c.hstage;
            double* st_n = st_rep + rstride * ns;
            if ((rc = hcheck(hipMemcpyAsync(st_rep, c.sc.rep, rstride * ns * sizeof(double), hipMemcpyDeviceToHost,
                                            c.st),
                             "copy")))
                return rc;
            if ((rc = hcheck(hipMemcpyAsync(st_n, c.sc.nrm2, ns * sizeof(double), hipMemcpyDeviceToHost, c.st),
                             "copy")))
                return rc;
            if ((rc = hcheck(hipStreamSynchronize(c.st), "arnoldi step"))) return rc;
            float ms = 0;
            if (hipEventElapsedTime(&ms, c.ev[0], c.ev[1]) == hipSuccess) c.t_sap += ms * 1e-3;
            ++steps;
            // a non-finite Hessenberg entry (an overflow in the preconditioner
            // or the operator) would otherwise read as a breakdown
            for (int k = 0; k < ns; ++k)
                for (size_t i = 0; i < 4 + 4 * (size_t)j; ++i)
                    if (!std::isfinite(st_rep[k * rstride + i]) || !std::isfinite(st_n[k]))
                        return fail(TM_ERR_NONFINITE, "non-finite value in the Arnoldi step %d (preconditioned vector)",
                                    steps);
            bool all_frozen = true;
            for (int k = 0; k < ns; ++k) {
                if (frozen[k]) continue;
                const double* rk = st_rep + rstride * k;  // beta, h, s, then (c_i, a_i) in the basis V
                zc* Hk = &Hraw[(size_t)k * (m + 1) * m];
                zc* gk = &gv[(size_t)k * (m + 1)];
                if (j > 0) {
                    // finish column j-1: w_{j-1} = V h + u_j / s_{j-1} with u_j = V c + beta v_j
                    const double beta = rk[0], sj = sprev[k];
                    gk[j - 1] = gsave[k];  // undo the provisional rotation of column j-1
                    for (int i = 0; i < j; ++i) Hk[i * m + j - 1] += zc(rk[4 + 4 * i], rk[4 + 4 * i + 1]) / sj;
                    if (beta == 0.0) {
                        // u_j lies in the span of v_0..v_{j-1}: column j-1 closes the Krylov space
                        Hk[j * m + j - 1] = 0.0;
                        commit(k, j - 1);
                        kdim[k] = j;
                        frozen[k] = 1;
                        continue;
                    }
                    Hk[j * m + j - 1] = beta / sj;
                    commit(k, j - 1);
                }
                ++out.iters[k];
                // provisional column j (its second projection comes with the next step):
                // w_j = V_{j-1} a + h v_j + u_{j+1} / s
                for (int i = 0; i < j; ++i) Hk[i * m + j] = zc(rk[4 + 4 * i + 2], rk[4 + 4 * i + 3]);
                Hk[j * m + j] = zc(rk[1], rk[2]);
                const double s = rk[3];
                const double hn = s > 0 ? std::sqrt(std::max(0.0, st_n[k])) / s : 0.0;
                Hk[(j + 1) * m + j] = hn;
                sprev[k] = s;
                gsave[k] = gk[j];
                commit(k, j);
                kdim[k] = j + 1;
                const bool done = std::abs(gk[j + 1]) <= tol[k] * bnorm[k] || hn == 0.0;
                if (done) frozen[k] = 1;
                all_frozen &= (bool)frozen[k];
            }
            jdone = j + 1;
            if (verbose()) {
                double worst = 0.0;
                int active = 0;
                for (int k = 0; k < ns; ++k) {
                    const zc* gk = &gv[(size_t)k * (m + 1)];
                    if (bnorm[k] > 0) worst = std::max(worst, std::abs(gk[kdim[k]]) / bnorm[k]);
                    active += !frozen[k];
                }
                std::fprintf(stderr, "[tm] %s step %d: max residual estimate %.3e, %d of %d systems active, sap %.3f s\n",
                             c.vp == P_F64 ? "fgmres" : "inner fgmres", steps, worst, active, ns, c.t_sap);
                std::fflush(stderr);
            }
            if (all_frozen) break;
        }
        // x += Z y, y = R^-1 g per system (zero beyond its Krylov dimension)
        bool by_estimate = trust_estimate;
        for (int k = 0; k < ns; ++k) by_estimate &= (bool)frozen[k];
        std::vector<double> yh((size_t)ns * jdone * 2, 0.0);
        for (int k = 0; k < ns; ++k) {
            const zc* Rk = &R[(size_t)k * (m + 1) * m];
            const zc* gk = &gv[(size_t)k * (m + 1)];
            // a zero pivot comes from a zero preconditioned direction: the columns from there on
            // add nothing, so the solution uses the ones before it
            int kd = kdim[k];
            for (int i = 0; i < kd; ++i)
                if (std::abs(Rk[i * m + i]) == 0.0) {
                    kd = i;
                    if (i == 0) stalled |= 1ull << k;
                    break;
                }
            std::vector<zc> y(kd);
            for (int i = kd - 1; i >= 0; --i) {
                zc t = gk[i];
                for (int q = i + 1; q < kd; ++q) t -= Rk[i * m + q] * y[q];
                y[i] = t / Rk[i * m + i];
            }
            for (int i = 0; i < kd; ++i) {
                yh[((size_t)k * jdone + i) * 2] = y[i].real();
                yh[((size_t)k * jdone + i) * 2 + 1] = y[i].imag();
            }
        }
        if (jdone > 0) {
            std::memcpy(c.hy, yh.data(), yh.size() * sizeof(double));
            if ((rc = hcheck(hipMemcpyAsync(c.sc.y, c.hy, yh.size() * sizeof(double), hipMemcpyHostToDevice, c.st),
                             "copy")))
                return rc;
            const SpinorBuf z0 = K.Zb(c, 0);
            const size_t zscale_stride = K.zstride / sizeof(float);
            out.accumulated = x_acc && x_zero && by_estimate;
            if (out.accumulated) {
                if ((rc = hcheck(blas_xupdate(P_F64, c.sp, vec_ref(*x_acc, V), vec_ref(z0, V), K.zstride,
                                              zscale_stride, jdone, c.sc.y, x_acc_zero, ns, V, c.st),
                                 "x update")))
                    return rc;
            } else if ((rc = hcheck(blas_xupdate(c.vp, c.sp, vec_ref(x, V), vec_ref(z0, V), K.zstride, zscale_stride,
                                                 jdone, c.sc.y, x_zero, ns, V, c.st),
                                    "x update"))) {
                return rc;
            }
        }
        if (by_estimate) {
            for (int k = 0; k < ns; ++k) {
                if (((skip >> k) & 1ull) || bnorm[k] == 0) continue;
                out.rel[k] = std::abs(gv[(size_t)k * (m + 1) + kdim[k]]) / bnorm[k];
                out.conv[k] = out.rel[k] <= tol[k] && !((stalled >> k) & 1ull);
            }
            return TM_OK;
        }
        x_zero = false;
        if ((rc = residual(c, rhs, x, false, V0, rn2.data(), bn2.data()))) return rc;
    }
    if (x_zero) {
        // no cycle ran: the solution is zero
        if (x_acc && !x_acc_zero)
            out.accumulated = true;
        else if ((rc = hcheck(blas_zero((x_acc ? *x_acc : x).data, internal_bytes(c.g, ns, x_acc ? P_F64 : c.vp),
                                        c.st),
                              "zero")))
            return rc;
        else if (x_acc)
            out.accumulated = true;
    }
    return TM_OK;
}

int carve_scratch(Ctx& c) {
    const int nblk = blas_blocks(c.g.V);
    const size_t nvals = (size_t)c.nsys * 2 * blas_max_vec();
    const size_t nrep = (size_t)c.nsys * (4 + 4 * blas_max_vec());
    const size_t ntri = (size_t)c.nsys * blas_max_vec() * blas_max_vec() * 2;
    const size_t doubles = 5 * c.nsys + 5 * nvals + nrep + c.nsys + ntri + nvals * nblk + 64;
    hipError_t e = c.ds->red.ensure(doubles * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "solver scratch");
    double* p = (double*)c.ds->red.ptr;
    c.sc.inv = p; p += c.nsys;
    c.sc.ones = p; p += c.nsys;
    c.sc.y = p; p += nvals;
    c.sc.res = p; p += 2 * c.nsys;
    c.sc.dots = p; p += 2 * nvals;
    c.sc.coef = p; p += 2 * nvals;
    c.sc.rep = p; p += (size_t)c.nsys * (4 + 4 * blas_max_vec());
    c.sc.nrm2 = p; p += c.nsys;
    c.sc.tri = p; p += (size_t)c.nsys * blas_max_vec() * blas_max_vec() * 2;
    c.sc.partials = p;
    const size_t stage = nrep + c.nsys + 32, hinv = c.nsys + 32, hy = nvals + 32;
    e = c.host.ensure(stage + hinv + hy);
    if (e != hipSuccess) return hip_fail(e, "pinned host buffer");
    c.hstage = c.host.p;
    c.hinv = c.host.p + stage;
    c.hy = c.host.p + stage + hinv;
    for (int k = 0; k < c.nsys; ++k) c.hinv[k] = 1.0;
    e = hipMemcpyAsync(c.sc.ones, c.hinv, c.nsys * sizeof(double), hipMemcpyHostToDevice, c.st);
    if (e == hipSuccess) e = hipStreamSynchronize(c.st);
    return e == hipSuccess ? TM_OK : hip_fail(e, "scratch init");
}


}  // namespace

// Largest group of systems whose workspace fits in free device memory.
int fit_group(DeviceState* ds, int nsys, int group, size_t per_sys, size_t fixed, size_t reusable) {
    int gsz = group > 0 ? std::min(group, nsys) : nsys;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return gsz;
    const size_t avail = (size_t)((double)(free_b + ds->solver.bytes + reusable) * 0.92);
    while (gsz > 1 && fixed + per_sys * (size_t)gsz > avail) gsz = (gsz + 1) / 2;
    return gsz;
}

}  // namespace tmsap

using namespace tmsap;

extern "C" {

void tm_solver_opts_default(tm_solver_opts* s) {
    if (!s) return;
    std::memset(s, 0, sizeof *s);
    s->form = TM_SOLVE_FLEXIBLE;
    s->restart = 20;
    s->max_iters = 2000;
    s->n_cycles = 4;
    s->mr_iters = 4;
    for (int a = 0; a < 4; ++a) s->block_dims[a] = 4;
    s->inner_tol = 1e-6;
    s->max_outer = 50;
    s->group = 0;
    s->x_in = 1;
}

int tm_fgmres_solve(const tm_geom* geom, const void* U, const void* b, void* x, double kappa, double c_sw, double tol,
                    const tm_solver_opts* so, const tm_opts* opts, tm_solve_report* report) {
    const auto t_start = std::chrono::steady_clock::now();
    int rc;
    if ((rc = check_geom(geom)) || (rc = check_opts(opts))) return rc;
    if (!so) return fail(TM_ERR_ARG, "solver options are NULL");
    if (!U || !b || !x) return fail(TM_ERR_ARG, "null pointer");
    if (b == x) return fail(TM_ERR_ARG, "b and x alias");
    if (opts->io != TM_IO_CANONICAL) return fail(TM_ERR_ARG, "tm_fgmres_solve takes canonical buffers");
    if (!(tol > 0) || !(kappa > 0) || !std::isfinite(c_sw)) return fail(TM_ERR_ARG, "bad tol, kappa or c_sw");
    if (so->restart < 1 || so->restart > blas_max_vec() - 1)
        return fail(TM_ERR_ARG, "restart must be in 1..%d", blas_max_vec() - 1);
    if (so->n_cycles < 1 || so->mr_iters < 0 || so->max_iters < 1) return fail(TM_ERR_ARG, "bad iteration counts");
    if (so->form != TM_SOLVE_FLEXIBLE && so->form != TM_SOLVE_DEFECT_CORRECTION) return fail(TM_ERR_ARG, "unknown form");
    const Prec sp = (Prec)opts->storage;
    const bool dc = so->form == TM_SOLVE_DEFECT_CORRECTION;
    if (dc && sp == P_F64) return fail(TM_ERR_PREC, "defect correction needs FP32/FP16/BF16 smoother storage");
    if (dc && !(so->inner_tol > 0 && so->inner_tol < 1)) return fail(TM_ERR_ARG, "inner_tol must be in (0, 1)");
    // block_dims all zero: the tuned shape for this problem if one is cached, else 4^4; with a
    // two-level handle its aggregates
    int bd[4], tuned_tile = 0;
    tm_mg* mg = so->mg;
    if (mg) {
        if (sp != P_F32) return fail(TM_ERR_PREC, "the two-level preconditioner needs FP32 storage");
        if (opts->sap_eo) return fail(TM_ERR_ARG, "the two-level preconditioner smooths without even-odd blocks");
        if ((rc = mg_matches(mg, geom))) return rc;
    }
    const bool bd_given = so->block_dims[0] | so->block_dims[1] | so->block_dims[2] | so->block_dims[3];
    if (mg)
        mg_block_dims(mg, bd);
    else if (bd_given)
        for (int a = 0; a < 4; ++a) bd[a] = so->block_dims[a];
    else if (!tune_lookup(geom, opts->storage, so->n_cycles, so->mr_iters, opts->sap_eo, bd, &tuned_tile))
        for (int a = 0; a < 4; ++a) bd[a] = 4;
    int tile[4];
    if ((rc = check_sap_blocks(geom, bd, tile))) return rc;
    if (!sap_supported(sp, sp, clover_prec_for(sp), sp == P_F64 ? P_F64 : P_F32))
        return fail(TM_ERR_PREC, "unsupported smoother precision");
    DeviceState* ds = device_state(&rc);
    if (!ds) return rc;
    hipStream_t st = (hipStream_t)opts->stream;
    Geo g = make_geo(geom, tile);
    const long long V = g.V;

    const GaugeDev *op64, *op32 = nullptr, *gs;
    if ((rc = get_gauge(ds, g, U, kappa, c_sw, P_F64, opts->gauge_tag, st, &op64))) return rc;
    if (dc && (rc = get_gauge(ds, g, U, kappa, c_sw, P_F32, opts->gauge_tag, st, &op32))) return rc;
    if (sp == P_F64)
        gs = op64;
    else if (sp == P_F32 && op32)
        gs = op32;
    else if ((rc = get_gauge(ds, g, U, kappa, c_sw, sp, opts->gauge_tag, st, &gs)))
        return rc;

    const Prec vp = dc ? P_F32 : P_F64;
    const int m = so->restart;
    // bytes per system: outer FP64 vectors (b, x, and r for defect correction) + Krylov space (+ r32, c32)
    const size_t b64 = internal_bytes(g, 1, P_F64);
    const size_t per_sys = (dc ? 3 : 2) * b64 + krylov_bytes(g, 1, m, vp, sp) +
                           (dc ? 2 * internal_bytes(g, 1, P_F32) : 0) + (mg ? mg_workspace_per_sys(mg) : 0);
    const int group = fit_group(ds, geom->nsys, so->group, per_sys, 0, mg ? mg_workspace_held(mg) : 0);

    Ctx c;
    c.ds = ds;
    c.st = st;
    c.g = g;
    c.n_cycles = so->n_cycles;
    c.mr_iters = so->mr_iters;
    c.sys_tile = opts->sys_tile > 0 ? opts->sys_tile : tuned_tile;
    c.eo = opts->sap_eo != 0;
    c.sap = gs;
    c.mg = mg;
    c.vp = vp;
    c.sp = sp;
    if ((rc = hcheck(hipEventCreate(&c.ev[0]), "event")) || (rc = hcheck(hipEventCreate(&c.ev[1]), "event"))) return rc;
    struct EvGuard {
        Ctx& c;
        ~EvGuard() {
            (void)hipEventDestroy(c.ev[0]);
            (void)hipEventDestroy(c.ev[1]);
        }
    } evguard{c};

    tm_solve_report rep;
    std::memset(&rep, 0, sizeof rep);
    int all_conv = 1;
    const size_t canon_sys = (size_t)V * 12 * 2 * sizeof(double);
    for (int g0 = 0; g0 < geom->nsys; g0 += group) {
        const int ns = std::min(group, geom->nsys - g0);
        c.nsys = ns;
        for (int k = 0; k < kMaxSys; ++k) c.mu[k] = k < ns ? geom->mu[g0 + k] : 0.0;
        size_t bytes = (dc ? 3 : 2) * internal_bytes(g, ns, P_F64) + krylov_bytes(g, ns, m, vp, sp) +
                       (dc ? 2 * internal_bytes(g, ns, P_F32) : 0);
        hipError_t h = ds->solver.ensure(bytes);
        if (h != hipSuccess) return hip_fail(h, "solver workspace");
        if ((rc = carve_scratch(c))) return rc;
        char* p = (char*)ds->solver.ptr;
        SpinorBuf bb = wrap_internal(p, g, ns, P_F64);
        p += internal_bytes(g, ns, P_F64);
        SpinorBuf xx = wrap_internal(p, g, ns, P_F64);
        p += internal_bytes(g, ns, P_F64);
        const char* bcan = (const char*)b + g0 * canon_sys;
        char* xcan = (char*)x + g0 * canon_sys;
        if ((h = ds->stats.ensure(256)) != hipSuccess) return hip_fail(h, "stats");
        unsigned* flag = (unsigned*)ds->stats.ptr + 2;
        if ((rc = hcheck(hipMemsetAsync(flag, 0, sizeof(unsigned), st), "memset"))) return rc;
        if ((rc = hcheck(launch_spinor_import(g, bb, bcan, flag, st), "import b"))) return rc;
        if (so->x_in && (rc = hcheck(launch_spinor_import(g, xx, xcan, flag, st), "import x"))) return rc;
        unsigned hflag = 0;
        if ((rc = hcheck(hipMemcpyAsync(&hflag, flag, sizeof hflag, hipMemcpyDeviceToHost, st), "copy"))) return rc;
        if ((rc = hcheck(hipStreamSynchronize(st), "import"))) return rc;
        if (hflag) return fail(TM_ERR_NONFINITE, "b or x holds NaN or Inf");

        // a zero starting vector (every system of the group) makes the first residual b itself;
        // without x_in the FP64 iterate starts as zeros
        bool x_zero = true;
        if (so->x_in) {
            if ((rc = hcheck(blas_norm2(P_F64, vec_ref(xx, V), c.sc.partials, c.sc.res, ns, V, st), "norm")))
                return rc;
            if ((rc = hcheck(hipMemcpyAsync(c.hstage, c.sc.res, ns * sizeof(double), hipMemcpyDeviceToHost, st),
                             "copy")))
                return rc;
            if ((rc = hcheck(hipStreamSynchronize(st), "norm"))) return rc;
            for (int k = 0; k < ns; ++k) x_zero &= c.hstage[k] == 0.0;
        }
        // without x_in the FP64 iterate is not written until the solve writes it (a zero start
        // never reads it; the first correction overwrites it)

        CoreResult res;
        if (!dc) {
            c.op = op64;
            c.op_compute = P_F64;
            Krylov K = carve_krylov(p, g, ns, m, vp, sp);
            std::vector<double> tols(ns, tol);
            if ((rc = fgmres_core(c, K, bb, xx, x_zero, tols.data(), so->max_iters, res))) return rc;
            for (int k = 0; k < ns; ++k) {
                rep.true_rel_res[g0 + k] = res.rel[k];
                rep.iters = std::max(rep.iters, res.iters[k]);
                rep.converged += res.conv[k];
                all_conv &= res.conv[k];
            }
        } else {
            SpinorBuf rr = wrap_internal(p, g, ns, P_F64);
            p += internal_bytes(g, ns, P_F64);
            SpinorBuf r32 = wrap_internal(p, g, ns, P_F32);
            p += internal_bytes(g, ns, P_F32);
            SpinorBuf c32 = wrap_internal(p, g, ns, P_F32);
            p += internal_bytes(g, ns, P_F32);
            Krylov K = carve_krylov(p, g, ns, m, vp, sp);
            std::vector<double> rn2(ns), bn2(ns);
            std::vector<int> iters(ns, 0);
            int outer = 0;
            bool done = false;
            bool xx_zero = x_zero;  // the FP64 iterate is the zero start (possibly not yet written)
            for (;;) {
                // FP64 residual of the current iterate, rounded once into the inner solve's FP32
                // right-hand side (b itself for a zero start: then that is converted from b)
                c.vp = P_F64;
                c.op = op64;
                c.op_compute = P_F64;
                const bool r_is_b = x_zero && outer == 0;
                if (r_is_b) {
                    if ((rc = hcheck(blas_norm2(P_F64, vec_ref(bb, V), c.sc.partials, c.sc.res, ns, V, st), "norm")))
                        return rc;
                    if ((rc = hcheck(hipMemcpyAsync(c.hstage, c.sc.res, ns * sizeof(double), hipMemcpyDeviceToHost,
                                                    st),
                                     "copy")))
                        return rc;
                    if ((rc = hcheck(hipStreamSynchronize(st), "norm"))) return rc;
                    for (int k = 0; k < ns; ++k) {
                        rn2[k] = bn2[k] = c.hstage[k];
                        if (!std::isfinite(rn2[k])) return fail(TM_ERR_NONFINITE, "non-finite residual of system %d", k);
                    }
                } else if ((rc = residual(c, bb, xx, false, rr, rn2.data(), bn2.data(), &r32))) {
                    return rc;
                }
                done = true;
                // stagnation: a correction that left every unconverged system's residual no
                // smaller (a preconditioner that returns zero) ends the loop unconverged
                bool stagnant = outer > 0;
                for (int k = 0; k < ns; ++k) {
                    const double rel = bn2[k] > 0 ? std::sqrt(rn2[k] / bn2[k]) : 0.0;
                    if (rel > tol && rel < rep.true_rel_res[g0 + k]) stagnant = false;
                    rep.true_rel_res[g0 + k] = rel;
                    done &= rel <= tol;
                }
                if (done) stagnant = false;
                int maxit = 0;
                for (int k = 0; k < ns; ++k) maxit = std::max(maxit, iters[k]);
                if (verbose()) {
                    double worst = 0.0;
                    for (int k = 0; k < ns; ++k) worst = std::max(worst, rep.true_rel_res[g0 + k]);
                    std::fprintf(stderr, "[tm] systems %d..%d outer %d: max true residual %.3e after %d iterations\n",
                                 g0, g0 + ns - 1, outer, worst, maxit);
                    std::fflush(stderr);
                }
                if (done || stagnant || outer >= so->max_outer || maxit >= so->max_iters) break;
                // inner FP32 solve of D c = r to inner_tol, then x += c
                if (r_is_b && (rc = hcheck(launch_spinor_convert(g, bb, r32, st), "convert"))) return rc;
                c.vp = P_F32;
                c.op = op32;
                c.op_compute = P_F32;
                // each system's own inner tolerance: inner_tol, relaxed to what its outer
                // tolerance still needs (never below 0.5 tol ||b_k|| / ||r_k||); a system that
                // has already converged is skipped (frozen in every restart cycle, its x left
                // as it is)
                std::vector<double> itol(ns, so->inner_tol);
                unsigned long long skip = 0;
                for (int k = 0; k < ns; ++k) {
                    if (rep.true_rel_res[g0 + k] <= tol) {
                        skip |= 1ull << k;
                        continue;
                    }
                    if (rn2[k] > 0 && bn2[k] > 0)
                        itol[k] = std::max(itol[k], 0.5 * tol * std::sqrt(bn2[k] / rn2[k]));
                    itol[k] = std::min(itol[k], 0.5);
                }
                if (verbose()) {
                    for (int k = 0; k < ns; ++k)
                        std::fprintf(stderr, "[tm]   system %d: true residual %.6e, inner tolerance %.3e%s\n",
                                     g0 + k, rep.true_rel_res[g0 + k], itol[k],
                                     ((skip >> k) & 1ull) ? " (converged, skipped)" : "");
                    std::fflush(stderr);
                }
                if ((rc = fgmres_core(c, K, r32, c32, true, itol.data(), so->max_iters - maxit, res, skip, true,
                                      &xx, xx_zero)))
                    return rc;
                for (int k = 0; k < ns; ++k) iters[k] += res.iters[k];
                if (!res.accumulated) {
                    // x += c, or x = c while x is still the zero start
                    const hipError_t h = xx_zero
                                             ? blas_scale(P_F32, P_F64, vec_ref(c32, V), c.sc.ones, vec_ref(xx, V), ns, V, st)
                                             : blas_accumulate(P_F64, P_F32, vec_ref(xx, V), vec_ref(c32, V), ns, V, st);
                    if ((rc = hcheck(h, "accumulate"))) return rc;
                }
                xx_zero = false;
                ++outer;
            }
            if (xx_zero && (rc = hcheck(blas_zero(xx.data, internal_bytes(g, ns, P_F64), st), "zero")))
                return rc;  // no correction was made: the solution is the zero start
            for (int k = 0; k < ns; ++k) {
                const bool ok = rep.true_rel_res[g0 + k] <= tol;
                rep.converged += ok;
                all_conv &= ok;
                rep.iters = std::max(rep.iters, iters[k]);
            }
            rep.outer = std::max(rep.outer, outer);
        }
        if ((rc = hcheck(launch_spinor_export(g, xx, xcan, st), "export x"))) return rc;
        if ((rc = hcheck(hipStreamSynchronize(st), "export"))) return rc;
    }
    for (int a = 0; a < 4; ++a) rep.block_dims[a] = bd[a];
    rep.sys_tile = c.sys_tile;
    rep.t_sap = c.t_sap;
    rep.sap_cycles = c.sap_cycles;
    rep.sap_sys_cycles = c.sap_sys_cycles;
    rep.group = group;
    rep.t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (report) *report = rep;
    return all_conv ? TM_OK : TM_NOT_CONVERGED;
}

}  // extern "C"
