"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic byte and flop model that
the roofline divides, and the reading of the committed counter summary."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    # the guard runs before torch or the library is imported
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_sap_byte_model_counts_links_clover_and_spinors():
    # per site of the swept colour: 4 links as two rows (4 x 12 reals), the clover's two Hermitian
    # 6x6 blocks (2 x 36 reals), and per system b and x read and x written (3 x 24 reals)
    for storage, rb in (("f64", 8), ("f32", 4)):
        for nsys in (1, 2, 12):
            assert bench.sap_bytes_per_site_cycle(storage, nsys) == (48 + 72) * rb + nsys * 3 * 24 * rb
    # 16-bit storage keeps the clover in FP32; FP16 spinors carry one FP32 scale per site
    assert bench.sap_bytes_per_site_cycle("bf16", 2) == 48 * 2 + 72 * 4 + 2 * 3 * 24 * 2
    assert bench.sap_bytes_per_site_cycle("f16", 2) == 48 * 2 + 72 * 4 + 2 * 3 * (24 * 2 + 4)
    # the 12-system half-sweep of 48^3x96 moves 20,893,925,376 bytes (half of the 10.6 M sites)
    V = 48 * 48 * 48 * 96
    assert bench.sap_bytes_per_site_cycle("f32", 12) * V // 2 == 20893925376


def test_sap_flop_model():
    # a hop: (1 -/+ gamma) projection 12 complex adds, U on two colour vectors (2 x (9 complex
    # multiplies + 6 complex adds)), lift 6 complex adds
    assert bench.HOP_FLOPS == 12 * 2 + 2 * (9 * 6 + 6 * 2) + 6 * 2
    # a zero-guess application: the first cycle forms no residual on colour 0 and only the halo
    # hops on colour 1, so it costs less than a steady cycle
    b1, f1 = bench.sap_application_model("f32", 6, 1, 4)
    b4, f4 = bench.sap_application_model("f32", 6, 4, 4)
    steady_b = bench.sap_bytes_per_site_cycle("f32", 6)
    steady_f = bench.sap_flops_per_site_cycle(6, 4)
    assert b4 - b1 == pytest.approx(3 * steady_b)
    assert f4 - f1 == pytest.approx(3 * steady_f)
    assert b1 < steady_b and f1 < steady_f


def test_traffic_summary_is_read_only_for_the_sources_it_was_taken_with(monkeypatch):
    path = os.path.join(ROOT, "profiles", bench.TRAFFIC_SUMMARIES[("k_sap_half_44", "48^3x96_12rhs_f32")])
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    want = float(kv["fetch_bytes_per_launch"]) * float(kv["fetch_factor"]) + \
        float(kv["write_bytes_per_launch"]) * float(kv["write_factor"])
    monkeypatch.setattr(bench, "sap_source_hash", lambda: kv["source_sha256"])
    assert bench.measured_traffic("k_sap_half_44", "48^3x96_12rhs_f32") == pytest.approx(want)
    # a changed kernel (another hash) or an unknown workload reports no traffic
    monkeypatch.setattr(bench, "sap_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic("k_sap_half_44", "48^3x96_12rhs_f32") is None
    assert bench.measured_traffic("k_sap_half_44", "32^3x64_pm_f32") is None

