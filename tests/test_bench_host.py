"""Host logic of bench.py without a GPU: the roofline fields are computed
from a launch's algorithmic bytes and time, and the counter-derived figures
(HBM bytes, VALU instructions, floating-point operations) are taken from
profiles/traffic.json only for the kernel source they were measured on."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def launch(ms, k=2, vb=4, nx=2048, ny=8192):
    nodes = nx * ny
    return dict(steps_per_launch=k, nodes=nodes, kernel_ms=ms, kernel="k", value_bytes=vb,
                bytes_per_launch=2 * 9 * vb * nodes)


def test_hbm_roofline_counts_the_launch_bytes_once_for_two_steps():
    r = launch(0.3)
    out = bench.roofline_of(r, 6000.0)
    assert out["bound"] == "hbm" and out["peak"] == 8000.0
    assert out["bytes_per_lu"] == 36
    assert out["achieved"] == pytest.approx(r["bytes_per_launch"] / 0.3e-3 / 1e9, rel=1e-4)
    assert out["frac"] == pytest.approx(out["achieved"] / 8000.0, abs=1e-4)
    assert out["frac_of_copy"] == pytest.approx(out["achieved"] / 6000.0, abs=1e-4)
    assert out["traffic"] is None and out["valu_issue"] is None
    assert bench.roofline_of(launch(0.3, k=1, vb=8), None)["bytes_per_lu"] == 144


def test_valu_ceiling_and_flop_rate():
    r = launch(0.2869)
    v = bench.valu_ceiling_of(r, 249.4, 283.6, "fp32")
    peak = 256 * 2.4e9 * 64 / 249.4 / 1e9
    got = 2 * 2048 * 8192 / 0.2869e-3 / 1e9
    assert v["bound"] == "alu" and v["peak"] == pytest.approx(peak, abs=0.05)
    assert v["achieved"] == pytest.approx(got, abs=0.05)
    assert v["flops"]["achieved_tflops"] == pytest.approx(got * 283.6 / 1e3, abs=0.01)
    assert v["flops"]["peak_tflops"] == 157.3 and v["flops"]["peak_tflops_unpacked"] == 78.6
    v64 = bench.valu_ceiling_of(launch(0.611, vb=8), 377.1, 345.1, "fp64")
    assert v64["flops"]["peak_tflops"] == 78.6 and "peak_tflops_unpacked" not in v64["flops"]
    assert bench.valu_ceiling_of(r, None) is None


def test_counter_figures_follow_the_kernel_source(monkeypatch):
    with open(bench.TRAFFIC_FILE) as fh:
        tr = json.load(fh)
    key = "shear/fp32dev/2"
    e = tr["per_launch"][key]
    monkeypatch.setattr(bench, "kernel_sha", lambda: tr["kernel_sha"])
    assert bench.traffic_of(key) == (e["bytes_per_launch"], e["ratio"], e["valu_insts_per_64_lu"],
                                     e["flops_per_lu"])
    assert bench.traffic_of("no/such/key") is None
    monkeypatch.setattr(bench, "kernel_sha", lambda: "0" * 16)
    assert bench.traffic_of(key) is None
    # the recorded counters belong to the kernel source as committed
    monkeypatch.undo()
    assert bench.kernel_sha() == tr["kernel_sha"]
