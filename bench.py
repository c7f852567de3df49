#!/usr/bin/env python3
"""Benchmark: SAP-smoothed twisted-mass solves on one MI355X.

A step is one pass of the whole hot path over one batch: gauge ingest and
clover build, RHS import, and the mixed-precision solve of every system to a
true relative residual of 1e-10 (FP64 residual loop around FP32 FGMRES + SAP),
with inputs resident in HBM when the timed region starts.

Printed on one JSON line:
  value            SAP-sweep algorithmic bytes moved per second of whole-step
                   wall time (GB/s)
  sap_kernel_GBps  the SAP half-sweep kernel's own algorithmic bandwidth over
                   the launches of the timed steps (event time on the solve's
                   stream), and its fraction of the 8 TB/s HBM peak
  sap_sweep_all_systems
                   the SAP half-sweep kernel with every system of the workload
                   in one launch, event-timed: GB/s, TFLOP/s, site-updates/s
  sap_sweeps_32^3x64
                   the same for the 32^3 x 64 configuration: the +-mu pair in
                   FP32 and one system in FP64 (the HBM-bound case)
  roofline         the dominant kernel (SAP half-sweep) against its binding
                   peak, with algorithmic bytes / flops per launch, and the
                   FP32 FMA rate measured on the device without packed FP32
                   (the ceiling these kernels can reach)
  solve            time per RHS of the batched mixed-precision solve vs the
                   plain FP64 single-RHS solve and the FP64 CG on the squared
                   even-odd reduced system, all to 1e-10 (the baselines' first
                   call, which allocates their workspaces, reported apart)
  cpu_baseline     the FP64 CPU oracle on bounded samples at 1 thread and all
                   host threads (operator, SAP cycle, an 8^4 solve), CPU model
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP64_VECTOR_PEAK_TFLOPS = 78.6
METRIC = "SAP sweep GB/s (% HBM peak); 12-rhs mixed vs 1-rhs FP64 time/rhs @1e-10"

WORKLOADS = {
    # name: dims (T,Z,Y,X), eps, kappa, mu, csw, systems (list of (spin, colour, mu sign)), storage
    "48^3x96_12rhs_f32": dict(dims=(96, 48, 48, 48), eps=0.6, kappa=0.1373, mu=0.0009, csw=1.5,
                              sources=[(s, c, 1) for s in range(4) for c in range(3)], storage="f32"),
    # solved as stated for this configuration: FP64 FGMRES(20) preconditioned directly by the FP32
    # SAP (the other workloads use defect correction, whose FP64 state is what fits in memory)
    "32^3x64_pm_f32": dict(dims=(64, 32, 32, 32), eps=0.6, kappa=0.1394, mu=0.001, csw=1.5,
                           sources=[(0, 0, 1), (0, 0, -1)], storage="f32", form="flexible", restart=20),
    # 12 point sources x both flavours; the canonical complex128 buffers of 24 systems (309 GB for b
    # and x) do not fit beside the solver, so the solves go in calls of one +-mu pair (chunk 2)
    "64^3x128_24sys_f16": dict(dims=(128, 64, 64, 64), eps=0.6, kappa=0.1373, mu=0.0009, csw=1.5,
                               sources=[(s, c, sg) for s in range(4) for c in range(3) for sg in (1, -1)],
                               storage="f16", chunk=2),
    "64^3x128_24sys_bf16": dict(dims=(128, 64, 64, 64), eps=0.6, kappa=0.1373, mu=0.0009, csw=1.5,
                                sources=[(s, c, sg) for s in range(4) for c in range(3) for sg in (1, -1)],
                                storage="bf16", chunk=2),
    "16^4_1rhs_f32": dict(dims=(16, 16, 16, 16), eps=0.5, kappa=0.1632, mu=0.003, csw=1.5,
                          sources=[(0, 0, 1)], storage="f32"),
}

BLOCK = (4, 4, 4, 4)
N_CYCLES, MR_ITERS = 4, 4
TOL = 1e-10

# Algorithmic work of one SAP cycle per site (every operand touched once):
#   links 4 x 12 reals (two rows, third rebuilt) + clover 72 reals, read once;
#   per system: b read (24 reals), x read (24) and x written (24).
LINK_REALS, CLOVER_REALS, SPINOR_REALS = 48, 72, 24
# Flops of one SAP cycle per site and system, 4^4 blocks, 4 MR steps:
#   residual b - D x: 8 hops x 168 + clover 552 + 48 = 1944
#   each MR step: D_BB rho with 6 in-block hops on average (6 x 168 + 552 + 24)
#   + <q,rho>, <q,q>, e += a rho, rho -= a q (336) = 1920
# where a hop is projection (24) + SU(3) x 2 columns (132) + reconstruction (12)
HOP_FLOPS = 24 + 132 + 12
RESID_FLOPS = 8 * HOP_FLOPS + 552 + 48
MR_FLOPS = 6 * HOP_FLOPS + 552 + 24 + 336
REAL_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
# Even-odd block solves (section 2.5), per site averaged over the two parities:
#   reduction r_o - D_oe D_ee^-1 r_e: D_ee^-1 on even sites (two 6x6 complex products, 552)
#   and the in-block hops on odd sites (6 x 168 + 24), half each = 792
#   each MR step on the reduced operator: even sites hops + D_ee^-1 (1560), odd sites hops +
#   clover + combine + dots and updates (1008 + 552 + 24 + 192 = 1776), half each = 1668
#   recovery e_e = D_ee^-1 (r_e - D_eo e_o): 1560 on even sites = 780
#   plus the site inverses read once per launch (144 reals per even site = 72 per site)
EO_REDUCE_FLOPS, EO_MR_FLOPS, EO_RECOVER_FLOPS = 792, 1668, 780
EO_INV_REALS = 72


def _real_bytes(storage):
    rb = REAL_BYTES[storage]
    cb = 4 if storage in ("f16", "bf16") else rb  # clover kept in FP32 for 16-bit storage
    sb = 4 if storage == "f16" else 0              # FP16 spinors carry one FP32 scale per site
    return rb, cb, sb


def sap_bytes_per_site_cycle(storage: str, nsys: int) -> float:
    """Steady-state cycle: links + clover once, per system b read, x read, x written."""
    rb, cb, sb = _real_bytes(storage)
    return LINK_REALS * rb + CLOVER_REALS * cb + nsys * 3 * (SPINOR_REALS * rb + sb)


def sap_application_model(storage: str, nsys: int, n_cycles: int, mr: int, eo: bool = False):
    """Algorithmic bytes and flops per site of one SAP application from a zero guess
    (the preconditioner): in the first cycle x is not read and the colour-0 sweep
    has no residual to form (r = b), the colour-1 sweep only the hops from colour 0
    (2 of 8 hops per site on average for 4^4 blocks)."""
    rb, cb, sb = _real_bytes(storage)
    shared = LINK_REALS * rb + CLOVER_REALS * cb + (EO_INV_REALS * cb if eo else 0)
    spin = SPINOR_REALS * rb + sb
    first = shared + nsys * 2 * spin               # b read, x written
    rest = shared + nsys * 3 * spin
    bytes_app = first + (n_cycles - 1) * rest
    mr_f = EO_REDUCE_FLOPS + mr * EO_MR_FLOPS + EO_RECOVER_FLOPS if eo else mr * MR_FLOPS
    first_f = 0.5 * (mr_f) + 0.5 * (2 * HOP_FLOPS + 24 + mr_f)  # two half-sweeps, per site of a cycle
    rest_f = RESID_FLOPS + mr_f
    flops_app = nsys * (first_f + (n_cycles - 1) * rest_f)
    return bytes_app, flops_app


def sap_flops_per_site_cycle(nsys: int, mr: int = MR_ITERS) -> float:
    return nsys * (RESID_FLOPS + mr * MR_FLOPS)


SAP_SOURCES = ("paper_1610_02370_amd/csrc/tm_sap.hip", "paper_1610_02370_amd/csrc/tm_device.h",
               "paper_1610_02370_amd/csrc/tm_internal.h", "paper_1610_02370_amd/csrc/tm_sap_index.h")


def sap_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in SAP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


# rocprofv3 counter summaries (FETCH_SIZE / WRITE_SIZE) by (kernel, workload)
TRAFFIC_SUMMARIES = {
    ("k_sap_half_44", "48^3x96_12rhs_f32"): "sap_half_44_48cube_x96_12rhs_f32_traffic.txt",
}


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of the SAP kernel from the committed rocprofv3 counter summary.

    The summary holds FETCH_SIZE and WRITE_SIZE averaged over the kernel's
    launches in the timed region, each scaled by the factor a plain copy of
    known size gives for the same counter, and the hash of the kernel's
    sources when the counters were taken; a changed kernel gives None.
    """
    name = TRAFFIC_SUMMARIES.get((kernel, workload))
    if name is None:
        return None
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != sap_source_hash():
        return None
    try:
        return float(kv["fetch_bytes_per_launch"]) * float(kv["fetch_factor"]) + \
            float(kv["write_bytes_per_launch"]) * float(kv["write_factor"])
    except (KeyError, ValueError):
        return None


def copy_probe(torch, nbytes: int = 1 << 30):
    """A plain elementwise kernel of known traffic (nbytes read, nbytes written) for counter calibration."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    log(f"copy probe: neg of {nbytes} bytes ({nbytes} read, {nbytes} written)")
    del src, dst
    torch.cuda.empty_cache()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_inputs(wl, torch, tm, synth):
    import numpy as np

    dims = wl["dims"]
    V = int(np.prod(dims))
    t0 = time.time()
    U = synth.gauge_field(dims, wl["eps"], seed=4 if dims == (96, 48, 48, 48) else 3)
    log(f"gauge field generated in {time.time() - t0:.1f}s ({U.nbytes / 1e9:.1f} GB)")
    Ud = torch.from_numpy(U).cuda()
    del U
    nsys = len(wl["sources"])
    chunk = wl.get("chunk") or nsys
    b = torch.zeros((chunk, V, 4, 3), dtype=torch.complex128, device="cuda")
    set_sources(b, wl["sources"][:chunk])
    mus = [sg * wl["mu"] for (_, _, sg) in wl["sources"]]
    return Ud, b, mus


def sap_sweep_phase(wl, Ud, mus, torch, tm, reps, storage=None):
    """SAP cycles over all systems in one launch per half-sweep, event-timed on the stream."""
    dims = wl["dims"]
    storage = storage or wl["storage"]
    nsys = len(mus)
    nbytes = tm.tm_spinor_bytes(dims, nsys, storage, layout_block=BLOCK)
    bi = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    xi = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    # b: Gaussian-like content through the canonical import (one system at a time keeps memory low)
    from paper_1610_02370_amd import synth

    V = int(torch.tensor(dims).prod())
    g = torch.from_numpy(synth.gaussian_spinor(dims, 1, seed=100)).cuda()
    for k in range(nsys):  # one system at a time keeps the canonical staging at one field
        tm.tm_spinor_import_range(dims, g, bi, nsys, k, storage=storage, layout_block=BLOCK)
    del g
    xi.zero_()
    stream = torch.cuda.current_stream()
    # warm-up (gauge ingest happens here, tag 1 keeps the copy)
    tm.tm_sap_smooth(dims, Ud, bi, xi, wl["kappa"], mus, wl["csw"], BLOCK, 1, MR_ITERS, storage=storage,
                     io="internal", gauge_tag=1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        tm.tm_sap_smooth(dims, Ud, bi, xi, wl["kappa"], mus, wl["csw"], BLOCK, 1, MR_ITERS, storage=storage,
                         io="internal", gauge_tag=1)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    launches = 2 * reps
    per_launch_s = ms * 1e-3 / launches
    bytes_launch = V / 2 * sap_bytes_per_site_cycle(storage, nsys)
    flops_launch = V / 2 * sap_flops_per_site_cycle(nsys)
    del bi, xi
    torch.cuda.empty_cache()
    gbps = bytes_launch / per_launch_s / 1e9
    tflops = flops_launch / per_launch_s / 1e12
    alu_peak = FP64_VECTOR_PEAK_TFLOPS if storage == "f64" else FP32_VECTOR_PEAK_TFLOPS
    return {
        "dims_TZYX": list(dims),
        "systems": nsys,
        "storage": storage,
        "kernel": sap_kernel_name(storage),
        "launches": launches,
        "ms_per_launch": per_launch_s * 1e3,
        "GBps": gbps,
        "hbm_frac": gbps / HBM_PEAK_GBPS,
        "TFLOPs": tflops,
        "alu_frac": tflops / alu_peak,
        "site_updates_per_s": V * nsys * reps / (ms * 1e-3),
        "bytes_per_launch": bytes_launch,
        "flops_per_launch": flops_launch,
    }


def sap_kernel_name(storage: str, eo: bool = False) -> str:
    if eo:
        return "k_sap_half_eo"
    if storage == "f64":
        return "k_sap_half"
    return "k_sap_half_44" if tuple(BLOCK) == (4, 4, 4, 4) else "k_sap_half_v2"


def small_lattice_sweeps(torch, tm, synth, reps):
    """SAP sweeps of the 32^3 x 64 configuration (eps 0.6, kappa 0.1394, mu +-0.001, c_sw 1.5):
    the +-mu pair in FP32 and one system in FP64, the cases whose sweep the HBM bound can limit."""
    wl = WORKLOADS["32^3x64_pm_f32"]
    U = synth.gauge_field(wl["dims"], wl["eps"], seed=3)
    Ud = torch.from_numpy(U).cuda()
    del U
    out = {}
    out["32^3x64_pm_f32"] = sap_sweep_phase(wl, Ud, [wl["mu"], -wl["mu"]], torch, tm, reps)
    tm.tm_gauge_release(Ud)
    out["32^3x64_1sys_f64"] = sap_sweep_phase(wl, Ud, [wl["mu"]], torch, tm, reps, storage="f64")
    tm.tm_gauge_release(Ud)
    del Ud
    torch.cuda.empty_cache()
    for k, v in out.items():
        log(f"SAP sweep {k}: {v['ms_per_launch']:.3f} ms/launch, {v['GBps']:.0f} GB/s "
            f"({100 * v['hbm_frac']:.1f}% of HBM), {v['TFLOPs']:.1f} TFLOP/s")
    return out


def set_sources(b, srcs):
    """Point sources: unit entries at site 0, spin s and colour c of each system."""
    b.zero_()
    for k, (s, c, _) in enumerate(srcs):
        b[k, 0, s, c] = 1.0


def solve_step(wl, Ud, b, mus, x, torch, tm, restart, group, eo=False, tag=0, form="defect_correction"):
    """Every system of the workload solved to TOL, in calls of b.shape[0] systems (point sources
    set in b at the start of each call); returns the worst status and the merged report.  All
    calls of the step pass gauge tag `tag`: with 0 each call rebuilds the gauge copies, with a tag
    new to this step the first call rebuilds them and the later calls reuse them."""
    chunk = b.shape[0]
    rc_all, merged = 0, None
    for c0 in range(0, len(mus), chunk):
        srcs = wl["sources"][c0:c0 + chunk]
        n = len(srcs)
        if chunk < len(mus):  # one call holds every source: b was set once, before the timed steps
            set_sources(b, srcs)
        # zero starting vector: x is output only
        rc, rep = tm.tm_fgmres_solve(wl["dims"], Ud, b[:n], x[:n], wl["kappa"], mus[c0:c0 + n], wl["csw"], TOL,
                                     storage=wl["storage"], form=form, restart=restart,
                                     n_cycles=N_CYCLES, mr_iters=MR_ITERS, block_dims=BLOCK, group=group,
                                     gauge_tag=tag, eo=eo, x_in=False)
        rc_all = max(rc_all, rc)
        if merged is None:
            merged = dict(rep)
            merged["true_rel_res"] = list(rep["true_rel_res"])
        else:
            for k in ("t_total", "t_sap", "sap_cycles", "sap_sys_cycles"):
                merged[k] += rep[k]
            for k in ("iters", "outer"):
                merged[k] = max(merged[k], rep[k])
            merged["group"] = min(merged["group"], rep["group"])
            merged["converged"] += rep["converged"]
            merged["true_rel_res"] += list(rep["true_rel_res"])
    return rc_all, merged


def timed_twice(fn, torch):
    """(cold, warm) wall times of two identical calls: the first also allocates the workspaces, the
    second is the steady state.  Both rebuild the gauge copies (gauge tag 0), as the timed
    mixed-precision step does."""
    times, res = [], None
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return times[0], times[1], res


def fp64_baseline(wl, Ud, torch, tm, restart=20):
    import numpy as np

    dims = wl["dims"]
    V = int(np.prod(dims))
    b = torch.zeros((1, V, 4, 3), dtype=torch.complex128, device="cuda")
    s, c, sg = wl["sources"][0]
    b[0, 0, s, c] = 1.0
    x = torch.zeros_like(b)

    def run():
        return tm.tm_fgmres_solve(dims, Ud, b, x, wl["kappa"], [sg * wl["mu"]], wl["csw"], TOL, storage="f64",
                                  form="flexible", restart=restart, n_cycles=N_CYCLES, mr_iters=MR_ITERS,
                                  block_dims=BLOCK, gauge_tag=0, x_in=False)

    cold, warm, (rc, rep) = timed_twice(run, torch)
    tm.tm_gauge_release(Ud)
    del b, x
    return {"s_per_rhs": warm, "s_per_rhs_cold": cold, "iters": rep["iters"], "restart": restart,
            "true_rel_res": rep["true_rel_res"][0], "status": rc}


def cg_baseline(wl, Ud, torch, tm):
    """FP64 CG on the squared even-odd reduced system (the paper's comparison solver), one point source."""
    import numpy as np

    dims = wl["dims"]
    V = int(np.prod(dims))
    b = torch.zeros((1, V, 4, 3), dtype=torch.complex128, device="cuda")
    s, c, sg = wl["sources"][0]
    b[0, 0, s, c] = 1.0
    x = torch.zeros_like(b)

    def run():
        x.zero_()
        return tm.tm_cg_solve(dims, Ud, b, x, wl["kappa"], [sg * wl["mu"]], wl["csw"], TOL, max_iters=100000,
                              gauge_tag=0)

    cold, warm, (rc, rep) = timed_twice(run, torch)
    tm.tm_gauge_release(Ud)
    del b, x
    return {"s_per_rhs": warm, "s_per_rhs_cold": cold, "iters": rep["iters"],
            "true_rel_res": rep["true_rel_res"][0], "status": rc}


# Two-level method (sections 2.3 - 2.6) with the library defaults (Table 1 where a two-level
# method has the parameter): 4^4 aggregates, 28 test vectors, 5 setup iterations, coarse twist
# 5.2 mu, coarse GMRES(100) to 0.1, 4 post-smoothing cycles of 3 MR steps.
MG_NVEC = 28


def two_level_phase(wl, Ud, torch, tm, restart):
    """Setup of the two-level method (seeded Gaussian starting vectors drawn on the GPU) and the
    same multi-RHS defect-correction solve preconditioned by it instead of SAP."""
    import numpy as np

    dims = wl["dims"]
    V = int(np.prod(dims))
    # the earlier legs' library workspaces (Krylov bases, gauge copies) are released first
    tm.tm_finalize()
    torch.cuda.empty_cache()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2024)
    v0 = torch.randn((MG_NVEC, V, 4, 3), dtype=torch.complex128, device="cuda", generator=gen)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mg = tm.MG(dims, Ud, wl["kappa"], wl["mu"], wl["csw"], v0, n_vec=MG_NVEC)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    del v0
    torch.cuda.empty_cache()
    log(f"two-level setup: {t_setup:.2f}s")
    nsys = len(wl["sources"])
    b = torch.zeros((nsys, V, 4, 3), dtype=torch.complex128, device="cuda")
    for k, (s, c, _) in enumerate(wl["sources"]):
        b[k, 0, s, c] = 1.0
    mus = [sg * wl["mu"] for (_, _, sg) in wl["sources"]]
    x = torch.zeros_like(b)
    # the first solve also builds the operator's gauge copies and the solver workspaces; the
    # second is the steady state that is reported
    times = []
    for _ in range(2):
        before = mg.info()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, rep = tm.tm_fgmres_solve(dims, Ud, b, x, wl["kappa"], mus, wl["csw"], TOL, storage="f32",
                                     form="defect_correction", restart=restart, mg=mg, gauge_tag=11, x_in=False)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"two-level solve: {times[-1]:.2f}s iters {rep['iters']} outer {rep['outer']} group {rep['group']} "
            f"max res {max(rep['true_rel_res']):.2e}")
    info = mg.info()
    apps = info["applications"] - before["applications"]
    mg.close()
    tm.tm_gauge_release(Ud)
    del b, x
    torch.cuda.empty_cache()
    dt = times[-1]
    return {"setup_s": t_setup, "s_per_rhs": dt / nsys, "first_call_s_per_rhs": times[0] / nsys,
            "iters": rep["iters"], "outer": rep["outer"], "group": rep["group"], "status": rc,
            "max_true_rel_res": max(rep["true_rel_res"]), "n_vec": MG_NVEC,
            "coarse_dims_TZYX": list(info["cdims"]), "applications": apps,
            "coarse_steps_per_application": (info["coarse_iters"] - before["coarse_iters"]) / max(1, apps),
            "coarse_share": (info["t_coarse"] - before["t_coarse"]) / dt}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _rate(fn, sites: int, min_s: float):
    """Site-updates per second of fn over at least min_s seconds (at least one call)."""
    n, t0 = 0, time.perf_counter()
    while True:
        fn()
        n += 1
        dt = time.perf_counter() - t0
        if dt >= min_s:
            return sites * n / dt, n, dt


def cpu_baseline(wl):
    """The FP64 CPU oracle on bounded samples, at one host thread and at all of them:
    operator applications and SAP cycles (4^4 blocks, 4 MR steps, one system) on a 16^4 lattice
    with the workload's eps / kappa / mu / c_sw; the same two rates on the 32^3 x 64 lattice with
    that configuration's parameters (all threads); and the FGMRES(20) + SAP solve to 1e-10 of the
    8^4 run with the 32^3 x 64 configuration's parameters (eps 0.6, kappa 0.1394, mu 0.001,
    c_sw 1.5, gauge seed 3, point source).  `value` is the all-thread SAP rate at 16^4 converted
    with the GPU value's byte model."""
    import numpy as np

    import oracle
    from paper_1610_02370_amd import synth

    dims = (16, 16, 16, 16)
    V = int(np.prod(dims))
    U = synth.gauge_field(dims, wl["eps"], seed=5)
    psi = synth.gaussian_spinor(dims, 1, seed=105)[0].ravel()
    op = oracle.Operator(dims, U, oracle.kappa_to_m(wl["kappa"]), wl["mu"], wl["csw"])
    all_threads = oracle.num_threads()
    rates = {}
    for th in (1, all_threads):
        oracle.set_num_threads(th)
        d_rate, _, _ = _rate(lambda: op.apply(psi), V, 1.0)
        s_rate, cyc, _ = _rate(lambda: op.sap(psi, BLOCK, 1, MR_ITERS), V, 2.0)
        rates[th] = {"dirac_site_updates_per_s": d_rate, "sap_cycle_site_updates_per_s": s_rate,
                     "sap_cycles_timed": cyc}
    oracle.set_num_threads(all_threads)
    c3 = WORKLOADS["32^3x64_pm_f32"]
    # the 32^3 x 64 lattice itself (all threads): one operator application, one SAP cycle
    V3 = int(np.prod(c3["dims"]))
    U3 = synth.gauge_field(c3["dims"], c3["eps"], seed=3)
    psi3 = synth.gaussian_spinor(c3["dims"], 1, seed=103)[0].ravel()
    op3 = oracle.Operator(c3["dims"], U3, oracle.kappa_to_m(c3["kappa"]), c3["mu"], c3["csw"])
    d3_rate, _, _ = _rate(lambda: op3.apply(psi3), V3, 1.0)
    s3_rate, cyc3, _ = _rate(lambda: op3.sap(psi3, BLOCK, 1, MR_ITERS), V3, 1.0)
    del U3, psi3, op3
    # the 8^4 solve (configuration 3's parameters)
    d8 = (8, 8, 8, 8)
    U8 = synth.gauge_field(d8, c3["eps"], seed=3)
    op8 = oracle.Operator(d8, U8, oracle.kappa_to_m(c3["kappa"]), c3["mu"], c3["csw"])
    b8 = np.zeros((int(np.prod(d8)), 4, 3), np.complex128)
    b8[0, 0, 0] = 1.0
    t0 = time.perf_counter()
    _, rep8 = op8.fgmres(b8.ravel(), TOL, restart=20, precond=True, bdims=BLOCK, n_cycles=N_CYCLES,
                         mr_iters=MR_ITERS)
    solve8_s = time.perf_counter() - t0
    nsys = len(wl["sources"])
    per_site_sys = sap_bytes_per_site_cycle(wl["storage"], nsys) / nsys
    rate = rates[all_threads]["sap_cycle_site_updates_per_s"]
    return {
        "value": rate * per_site_sys / 1e9,
        "unit": "GB/s",
        "cores": all_threads,
        "kind": "oracle",
        "sample": f"SAP cycles (4^4 blocks, {MR_ITERS} MR steps, 1 system, FP64) on a 16^4 lattice with the "
                  f"workload's eps/kappa/mu/c_sw, {all_threads} threads; bytes per site-update from the GPU "
                  f"value's algorithmic model ({per_site_sys:.0f} B per site and system per cycle)",
        "cpu_model": cpu_model(),
        "threads": {"1": rates[1], str(all_threads): rates[all_threads]},
        "site_updates_per_s": rate,
        "lattice_32^3x64": {"dirac_site_updates_per_s": d3_rate, "sap_cycle_site_updates_per_s": s3_rate,
                            "sap_cycles_timed": cyc3, "threads": all_threads},
        "solve_8^4_cfg3_params": {"seconds": solve8_s, "iters": rep8["iters"],
                                  "true_rel_res": rep8["true_rel_res"], "threads": all_threads},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    # one untimed step first: the solver's workspaces (about 170 GB) are allocated there, and an
    # allocation right after another process released device memory can wait seconds for it
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="48^3x96_12rhs_f32", choices=sorted(WORKLOADS))
    ap.add_argument("--sap-reps", type=int, default=10)
    ap.add_argument("--restart", type=int, default=None,
                    help="FGMRES restart length (default: the workload's, else 8)")
    ap.add_argument("--form", choices=["defect_correction", "flexible"], default=None,
                    help="solver form (default: the workload's, else defect_correction)")
    ap.add_argument("--group", type=int, default=0)
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the SAP sweeps (every system of the workload in one launch; 32^3x64 +-mu FP32 and "
                         "1-system FP64)")
    ap.add_argument("--no-fp64-baseline", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cg-baseline", action="store_true")
    ap.add_argument("--no-two-level", action="store_true", help="skip the two-level method's setup and solve")
    ap.add_argument("--two-level-only", action="store_true",
                    help="only the two-level method's setup and solves (profiling)")
    ap.add_argument("--sweep-only", action="store_true", help="only the all-systems SAP sweep (profiling)")
    ap.add_argument("--eo", action="store_true",
                    help="even-odd preconditioned SAP block solves (section 2.5) instead of MR on the full block")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 1 GiB elementwise kernel before the timed region (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1610_02370_amd as tm
    from paper_1610_02370_amd import synth

    wl = WORKLOADS[args.workload]
    if args.restart is None:
        args.restart = wl.get("restart", 8)
    form = args.form or wl.get("form", "defect_correction")
    torch.cuda.set_device(0)
    Ud, b, mus = make_inputs(wl, torch, tm, synth)
    nsys = len(mus)
    dims = wl["dims"]
    V = int(torch.tensor(dims).prod())
    log(f"workload {args.workload}: V={V} systems={nsys} storage={wl['storage']}")

    if args.copy_probe:
        copy_probe(torch)

    if args.two_level_only:
        del b
        print(json.dumps({"two_level": two_level_phase(wl, Ud, torch, tm, args.restart)}), flush=True)
        return

    sweep, small_sweeps = None, None
    if not args.no_sweep or args.sweep_only:
        sweep = sap_sweep_phase(wl, Ud, mus, torch, tm, args.sap_reps)
        log(f"SAP sweep ({nsys} systems per launch): {sweep['ms_per_launch']:.3f} ms/launch, "
            f"{sweep['GBps']:.0f} GB/s, {sweep['TFLOPs']:.1f} TFLOP/s")
        tm.tm_gauge_release(Ud)
        if args.sweep_only:
            print(json.dumps({"sap_sweep": sweep}), flush=True)
            return
        if args.workload == "48^3x96_12rhs_f32":
            small_sweeps = small_lattice_sweeps(torch, tm, synth, args.sap_reps)

    b_chunk = b.shape[0]
    x = torch.zeros_like(b)
    # a step solved in several calls builds the gauge copies once, in its first call (one tag per
    # step, new each step); a step of one call rebuilds them in it (tag 0)
    chunked = b_chunk < nsys
    step_tag = (lambda k: 1000 + k) if chunked else (lambda k: 0)
    for w in range(args.warmup):
        rc, rep = solve_step(wl, Ud, b, mus, x, torch, tm, args.restart, args.group, args.eo, step_tag(w), form)
        log(f"warmup {w}: status {rc} iters {rep['iters']} outer {rep['outer']} t {rep['t_total']:.2f}s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for s in range(args.steps):
        rc, rep = solve_step(wl, Ud, b, mus, x, torch, tm, args.restart, args.group, args.eo,
                             step_tag(args.warmup + s), form)
        reps.append((rc, rep))
        log(f"step {s}: status {rc} iters {rep['iters']} outer {rep['outer']} group {rep['group']} "
            f"sap {rep['t_sap']:.2f}s total {rep['t_total']:.2f}s max res {max(rep['true_rel_res']):.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ok = all(rc == 0 for rc, _ in reps)
    if chunked:  # the baselines below start from no cached gauge copy, as after tag-0 steps
        tm.tm_gauge_release(Ud)

    # SAP launches of the timed region: every application is N_CYCLES cycles from a
    # zero guess over one group of systems; t_sap is event time on the solve's stream.
    t_sap = sum(r["t_sap"] for _, r in reps)
    sap_cycles = sum(r["sap_cycles"] for _, r in reps)
    sys_cycles = sum(r["sap_sys_cycles"] for _, r in reps)
    group = reps[0][1]["group"]
    apps = sap_cycles // N_CYCLES
    b_shared, f_shared = sap_application_model(wl["storage"], 0, N_CYCLES, MR_ITERS, args.eo)
    b_one, f_one = sap_application_model(wl["storage"], 1, N_CYCLES, MR_ITERS, args.eo)
    sys_apps = sys_cycles / N_CYCLES
    sap_bytes = V * (b_shared * apps + (b_one - b_shared) * sys_apps)
    sap_flops = V * (f_one - f_shared) * sys_apps
    launches = 2 * sap_cycles
    per_launch_s = t_sap / launches
    value = sap_bytes / wall / 1e9
    del x, b
    torch.cuda.empty_cache()

    # FGMRES(20) in FP64 does not fit next to 64^3 x 128 inputs: restart 8 there
    fp64 = None if args.no_fp64_baseline else fp64_baseline(wl, Ud, torch, tm,
                                                            restart=8 if V > 20_000_000 else 20)
    if fp64:
        log(f"FP64 1-RHS solve: {fp64['s_per_rhs']:.2f}s (first call {fp64['s_per_rhs_cold']:.2f}s) "
            f"iters {fp64['iters']} res {fp64['true_rel_res']:.2e}")
    cg = None if args.no_cg_baseline else cg_baseline(wl, Ud, torch, tm)
    if cg:
        log(f"FP64 CG (even-odd normal equations) 1-RHS: {cg['s_per_rhs']:.2f}s (first call "
            f"{cg['s_per_rhs_cold']:.2f}s) iters {cg['iters']} res {cg['true_rel_res']:.2e}")
    two = None
    if not args.no_two_level and wl["storage"] == "f32":
        two = two_level_phase(wl, Ud, torch, tm, args.restart)
    if two and cg:
        two["speedup_per_rhs_over_cg"] = cg["s_per_rhs"] / two["s_per_rhs"]
    if two and fp64:
        two["speedup_per_rhs_over_fp64_1rhs"] = fp64["s_per_rhs"] / two["s_per_rhs"]
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl)
    if cpu:
        log(f"CPU oracle: {cpu['value']:.3f} GB/s-equivalent on {cpu['cores']} threads")

    ms_per_step = wall / args.steps * 1e3
    t_rhs = wall / args.steps / nsys
    achieved_gbps = sap_bytes / t_sap / 1e9
    achieved_tflops = sap_flops / t_sap / 1e12
    kernel = sap_kernel_name(wl["storage"], args.eo)
    traffic = measured_traffic(kernel, args.workload)
    if wl["storage"] != "f64":
        # the FP32 vector rate these kernels can reach (no packed FP32), measured on this device
        fma = tm.tm_probe_fp32_fma()
        log(f"FP32 FMA probe: {fma:.1f} TFLOP/s")
        roof = {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                "measured_fp32_fma_tflops": fma, "frac_of_measured_fma": achieved_tflops / fma,
                "kernel": kernel, "launches": launches, "avg_launch_ms": per_launch_s * 1e3,
                "flops_per_launch": sap_flops / launches, "bytes_per_launch": sap_bytes / launches,
                "hbm_GBps": achieved_gbps, "hbm_frac": achieved_gbps / HBM_PEAK_GBPS}
    else:
        roof = {"bound": "hbm", "achieved": achieved_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved_gbps / HBM_PEAK_GBPS, "traffic": traffic, "kernel": kernel,
                "launches": launches, "avg_launch_ms": per_launch_s * 1e3, "bytes_per_launch": sap_bytes / launches}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": wl["storage"],
        "data": "synthetic",
        "config": {"workload": args.workload, "dims_TZYX": list(dims), "systems": nsys, "block": list(BLOCK),
                   "n_cycles": N_CYCLES, "mr_iters": MR_ITERS, "block_solve": "even-odd MR" if args.eo else "MR",
                   "tol": TOL, "solver_form": form, "restart": args.restart, "systems_per_call": b_chunk,
                   "group": group, "parallelism": "single GPU"},
        "converged": ok,
        "sap_kernel_GBps": achieved_gbps,
        "sap_kernel_hbm_frac": achieved_gbps / HBM_PEAK_GBPS,
        "sap": {"GBps": achieved_gbps, "hbm_frac": achieved_gbps / HBM_PEAK_GBPS, "TFLOPs": achieved_tflops,
                "site_updates_per_s": V * sys_cycles / t_sap, "share_of_step": t_sap / wall},
        "sap_sweep_all_systems": sweep,
        "sap_sweeps_32^3x64": small_sweeps,
        "solve": {"s_per_rhs_mixed": t_rhs, "iters": max(r["iters"] for _, r in reps),
                  "outer": max(r["outer"] for _, r in reps),
                  "max_true_rel_res": max(max(r["true_rel_res"]) for _, r in reps),
                  "s_per_rhs_fp64_1rhs": fp64["s_per_rhs"] if fp64 else None,
                  "s_per_rhs_fp64_1rhs_first_call": fp64["s_per_rhs_cold"] if fp64 else None,
                  "fp64_restart": fp64["restart"] if fp64 else None,
                  "fp64_iters": fp64["iters"] if fp64 else None,
                  "speedup_per_rhs": (fp64["s_per_rhs"] / t_rhs) if fp64 else None,
                  "s_per_rhs_cg_fp64": cg["s_per_rhs"] if cg else None,
                  "s_per_rhs_cg_fp64_first_call": cg["s_per_rhs_cold"] if cg else None,
                  "cg_iters": cg["iters"] if cg else None,
                  "speedup_per_rhs_over_cg": (cg["s_per_rhs"] / t_rhs) if cg else None},
        "two_level": two,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
