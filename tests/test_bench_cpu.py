"""Host logic of bench.py: the single-GPU refusal, the algorithmic bytes
behind the roofline, the kernel names it looks the recorded traffic up by,
and the rule that recorded traffic counts only for the sources it was taken
on.  No GPU is touched."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def bench():
    sys.path.insert(0, ROOT)
    import bench as b
    return b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""          # no JSON line for a run that did not happen


def test_algorithmic_bytes_per_site_update(bench):
    # 2 species x Q populations, each read once and written once
    assert bench.b_alg(19, 8) == 608 and bench.b_alg(19, 4) == 304
    assert bench.b_alg(9, 8) == 288 and bench.b_alg(9, 4) == 144


def test_repeat_summary_keeps_the_timed_sample_first(bench):
    """The timed region's step time comes first; the median and the spread
    (max - min over the median) cover it and the later samples."""
    r = {"kernel_ms": 2.20, "repeats_ms": [2.18, 2.19, 2.30, 2.21]}
    s = bench.repeat_summary(r)
    assert s["samples"] == 5 and s["kernel_ms"][0] == 2.2
    assert s["median_ms"] == 2.2
    assert s["spread"] == pytest.approx((2.30 - 2.18) / 2.20, abs=1e-4)
    assert bench.repeat_summary({"kernel_ms": 1.0, "repeats_ms": []}) == {
        "samples": 1, "kernel_ms": [1.0], "median_ms": 1.0, "spread": 0.0}


def test_tuned_kernels_have_recorded_traffic(bench):
    """The kernels bench.py times on the 256^3 workload (from the autotune
    table) are the ones whose counters profiles/traffic.json holds, under the
    names rocprofv3 reports; a retune that changes them needs new counters."""
    from paper_1112_5547_amd import autotune
    table = autotune.load()
    t = json.load(open(bench.TRAFFIC_JSON))
    assert t["sources_sha256"] == bench.kernel_sources_sha()
    for prec in ("fp64", "fp32_shifted"):
        for forcing, trt in (("shift", False), ("guo", False), ("shift", True)):
            kern = autotune.lookup(19, 256, 256, 256, prec, table, forcing)
            name = bench.kernel_symbol(kern, prec, forcing, trt)
            assert name in t["kernels"], name
            e = t["kernels"][name]
            alg = bench.b_alg(19, 8 if prec == "fp64" else 4) * 256 ** 3 / 2
            # reads and writes each at least their algorithmic share
            assert e["read_bytes"] >= 0.99 * alg and e["write_bytes"] >= 0.99 * alg


def test_traffic_is_null_for_other_sources(bench, monkeypatch):
    name = "sc::k_step_fused<19, sc::PF64, 64, 8>"
    gbps, nbytes = bench.traffic_for(name, 2.25)
    assert gbps is not None and nbytes > bench.b_alg(19, 8) * 256 ** 3
    assert abs(gbps - nbytes / 2.25e-3 / 1e9) < 1e-6
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda: "0" * 64)
    assert bench.traffic_for(name, 2.25) == (None, None)


def test_record_traffic_scales_by_the_copy_kernel(bench, tmp_path, monkeypatch):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) are scaled so that the copy
    kernel of known size reads and writes exactly its bytes."""
    def write(path, rows):
        with open(path, "w", newline="") as fh:
            w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Value"])
            w.writeheader()
            for k, v in rows:
                w.writerow({"Kernel_Name": k, "Counter_Value": v})
    copy_kib = bench.COPY_BYTES / 1024.0
    step = "void sc::k_step_fused<19, sc::PF64, 64, 8>(sc::StepParams)"
    write(tmp_path / "f.csv", [("sc::k_copy(unsigned long*)", copy_kib / 2),
                               (step, 1000.0), (step, 3000.0)])
    write(tmp_path / "w.csv", [("sc::k_copy(unsigned long*)", copy_kib), (step, 500.0)])
    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(tmp_path / "traffic.json"))
    bench.record_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    t = json.load(open(tmp_path / "traffic.json"))
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    e = t["kernels"]["sc::k_step_fused<19, sc::PF64, 64, 8>"]
    assert e["read_bytes"] == pytest.approx(2000.0 * 1024 * 2.0)     # mean of the dispatches
    assert e["write_bytes"] == pytest.approx(500.0 * 1024)
    assert t["sources_sha256"] == bench.kernel_sources_sha()
