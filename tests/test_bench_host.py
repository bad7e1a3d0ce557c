"""Host logic of the benchmark (no GPU): the roofline's canonical cost and
peaks, the kernel's own count of shared stencil rows, and the lookup of HBM
traffic records.

The canonical cost is the one the scope table states for the step: FP32
2,750 + 13,730 K flops and FP64 150 K + 30 flops per node-update (K the mean
predictor-corrector gathers), about 30.2 k FP32 flops at K = 2, against the
algorithmic 304 B (FP32-mixed) and 560 B (FP64) of HBM traffic per node.
"""
import math

import pytest

import bench
from paper_2405_11489_amd import workloads


def _launch(ms, kbar):
    return {"step_kernel_ms": ms, "kbar": kbar}


def test_canonical_fp32_roofline():
    N, k, ms = 1_000_000, 2.0, 1.0
    r = bench.roofline(_launch(ms, k), N, "fp32", 4, 16, 0, "kernel", None)
    assert r["flops_fp32_per_launch"] / N == pytest.approx(30_210)  # about 30.2 k at K = 2
    assert r["flops_fp64_per_launch"] / N == pytest.approx(330)
    # FP64 flops weighted by the ratio of the FP32 and FP64 vector peaks
    expect = (30_210 + 330 * 157.3 / 78.6) * N / (ms * 1e-3) / 1e12
    assert r["achieved"] == pytest.approx(expect)
    assert r["peak"] == 157.3 and r["frac"] == pytest.approx(expect / 157.3)
    assert r["frac_nonpacked"] == pytest.approx(expect / 78.6)
    assert r["hbm_bytes_algorithmic_per_launch"] == 304 * N
    assert r["bound"] == "alu" and r["traffic"] is None


def test_canonical_fp64_roofline():
    N, k, ms = 262_144, 3.0, 0.36
    r = bench.roofline(_launch(ms, k), N, "fp64", 4, 16, 0, "kernel", 123.0)
    per_node = 2_750 + 13_730 * k + 30 + 150 * k  # every flop in FP64
    assert r["flops_fp64_per_launch"] == pytest.approx(per_node * N)
    assert r["peak"] == 78.6
    assert r["frac"] == pytest.approx(per_node * N / (ms * 1e-3) / 1e12 / 78.6)
    assert r["hbm_bytes_algorithmic_per_launch"] == 560 * N
    assert r["traffic"] == 123.0


@pytest.mark.parametrize("T,rows", [(0.04, 5), (1.0, 9), (16.0, 16)])
def test_shared_rows_of_a_uniform_flow(T, rows):
    """Rows of the union of the four row stencils of an x-component (cubic
    stencil): 5 at sqrt T = 0.2 (the cold headline), 9 at sqrt T = 1, and at
    most the 16 rows of four separate stencils."""
    w = workloads.fourier_modes(n=8, ny=8, mach=0.0, amplitude=0.0, T0=T)
    assert bench.shared_rows_mean(w, 4) == rows


def test_own_count_shares_the_x_pass():
    canon = 13_730
    per_velocity = bench.flops_per_iter(4)
    shared = [bench.flops_per_iter(4, 16, r) for r in (5.0, 9.0, 16.0)]
    assert shared[0] < shared[1] < shared[2]
    assert shared[0] < 0.5 * canon          # the headline's five-row unions
    assert per_velocity < canon and math.isfinite(per_velocity)


def test_traffic_record_lookup(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k.md").write_text(
        "text\n"
        "traffic-record: kernel=step_tiled_kernel<float,4,0,D2Q16,8,8> precision=fp32 "
        "workload=wl sources_sha256=abc fetch_kib=1 write_kib=2 fetch_factor=0.5 "
        "write_factor=1.0 bytes_per_launch=12345\n"
        "traffic-record: kernel=step_tiled_kernel<float,4,0,D2Q16,8,8> precision=fp32 "
        "workload=wl sources_sha256=old bytes_per_launch=999\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    k = "step_tiled_kernel<float,4,0,D2Q16,8,8>"
    assert bench.traffic_record(k, "fp32", "wl") == 12345.0
    assert bench.traffic_record(k, "fp64", "wl") is None
    assert bench.traffic_record(k, "fp32", "other") is None
    assert bench.traffic_record("step_tiled_kernel<float,4,0,D2Q16,32,8>", "fp32", "wl") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "new")  # sources changed
    assert bench.traffic_record(k, "fp32", "wl") is None


def test_committed_records_name_the_headline_kernel():
    """profiles/ holds a record for the headline kernel on the 2048^2
    quadrants (whether it matches the current sources is checked by bench.py
    at run time, which reports null traffic otherwise)."""
    import os
    found = False
    for name in os.listdir(os.path.join(bench.ROOT, "profiles")):
        with open(os.path.join(bench.ROOT, "profiles", name)) as fh:
            for line in fh:
                if (line.startswith("traffic-record:")
                        and "kernel=step_tiled_kernel<float,4,0,D2Q16,8,8>" in line
                        and "workload=riemann_quadrants_2048x2048" in line):
                    found = True
    assert found
