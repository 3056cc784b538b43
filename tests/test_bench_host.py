"""Host logic of bench.py (no GPU): the algorithmic bytes of the roofline,
the summary of the rocprofv3 counter passes, the check that a stored traffic
figure belongs to the current kernel sources, and the refusal of more than
one GPU."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_per_update():
    # 8 links in, g(x) in and out, the neighbouring g once: 11 matrices
    assert bench.fixed_site_bytes(3) == 11 * 96 == 1056   # FP64-12
    assert bench.fixed_site_bytes(2) == 11 * 48 == 528    # FP32-12
    assert bench.fixed_site_bytes(0) == 11 * 144          # FP64-18
    assert bench.fixed_site_bytes(4) == 8 * 72 + 3 * 96   # split links, FP64-12 g


def _write_counters(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_summary_groups_dispatches_by_variant(tmp_path, monkeypatch):
    """Synthetic counter passes: a 1 GiB copy calibrates each counter, and the
    plain fixed-link dispatches of each (format, lanes, layout) group are
    assigned to the variants in the order the traffic run issues them, six
    per variant."""
    dims = (64, 64, 64, 64)
    Vh = 64 ** 4 // 2
    per = 2 * (bench.TRAFFIC_FIXED_SWEEPS - 1)
    fetch_kib_copy, write_kib_copy = 524288.0, 1048576.0   # 2 KiB and 1 KiB per counter unit
    fetch_rows = [("__amd_rocclr_copyBuffer", fetch_kib_copy)]
    write_rows = [("__amd_rocclr_copyBuffer", write_kib_copy)]
    expect = {}
    for fmt, variants in bench.TRAFFIC_FIXED_VARIANTS.items():
        for k, (lanes, block, order, layout) in enumerate(variants):
            # a distinct reading per variant: (1 + k / 100) x the algorithmic bytes
            alg = Vh * bench.fixed_site_bytes(fmt)
            fetch = 0.9 * alg * (1 + k / 100) / 2048.0
            write = 0.1 * alg * (1 + k / 100) / 1024.0
            rec = "true" if layout else "false"
            name = f"void lgf::fixed_sweep_kernel<{fmt}, {lanes}, false, 0, 0, {rec}>(...)"
            fetch_rows += [(name, fetch)] * per
            write_rows += [(name, write)] * per
            # the reunitarizing last sweep of the chunk is not a plain launch
            post1 = f"void lgf::fixed_sweep_kernel<{fmt}, {lanes}, false, 1, 0, {rec}>(...)"
            fetch_rows.append((post1, 1e9))
            write_rows.append((post1, 1e9))
            expect[bench.fixed_traffic_key(fmt, lanes, block, order, layout, dims)] = 1 + k / 100
    _write_counters(str(tmp_path / "fetch"), "FETCH_SIZE", fetch_rows)
    _write_counters(str(tmp_path / "write"), "WRITE_SIZE", write_rows)
    out_file = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out_file))
    bench.summarize_traffic(str(tmp_path / "fetch"), str(tmp_path / "write"), dims, "synthetic")
    t = json.loads(out_file.read_text())
    assert t["source_sha"] == bench.kernel_source_sha()
    assert t["calibration"]["FETCH_SIZE"]["bytes_per_counter_unit"] == pytest.approx(2048.0)
    assert t["calibration"]["WRITE_SIZE"]["bytes_per_counter_unit"] == pytest.approx(1024.0)
    for key, ratio in expect.items():
        e = t["kernels"][key]
        assert e["fetch_size_dispatches"] == per and e["write_size_dispatches"] == per, key
        assert e["hbm_over_algorithmic"] == pytest.approx(ratio, rel=1e-12), key
    key = next(iter(expect))
    assert bench.measured_traffic(key) == pytest.approx(t["kernels"][key]["hbm_bytes_per_launch"])
    # a figure taken on other kernel sources is never reported
    t["source_sha"] = "0" * 16
    out_file.write_text(json.dumps(t))
    assert bench.measured_traffic(key) is None


def test_committed_traffic_summary_covers_the_step_variants():
    """The committed counter summary was taken on the current kernel sources
    and holds every FP64-12 and split-storage variant the autotuner may pick
    on the 64^4 lattice (2 lanes, each workgroup size, the blocked order,
    both link layouts)."""
    t = json.load(open(bench.TRAFFIC_FILE))
    assert t["source_sha"] == bench.kernel_source_sha()
    for fmt in (3, 4):
        for block in (64, 128, 256):
            for layout in (0, 1):
                key = bench.fixed_traffic_key(fmt, 2, block, 2, layout, (64, 64, 64, 64))
                e = t["kernels"][key]
                assert 1.0 <= e["hbm_over_algorithmic"] < 1.10, (key, e["hbm_over_algorithmic"])


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_mixed_bulk_summary():
    """The mixed form's bulk sweep: 528 B per FP32-12 update over the launch
    time, its fraction of 8 TB/s and the site updates against the FP64 sweep."""
    Vh = 64 ** 4 // 2
    m = bench.mixed_bulk_summary(2, (1, 128, 0, 1), Vh, 0.8, 1.6)
    assert m["bytes_per_site_update"] == 528
    assert m["site_updates_per_s"] == pytest.approx(Vh / 0.8e-3)
    assert m["GBs"] == pytest.approx(Vh * 528 / 0.8e-3 / 1e9, abs=0.05)
    assert m["frac_of_8TBs"] == pytest.approx(m["GBs"] / 8000.0, abs=1e-4)
    assert m["site_updates_vs_fp64_sweep"] == 2.0
    assert "lanes/site 1" in m["kernel"] and "per-site link records" in m["kernel"]


def test_batched_summary():
    """The line's batched object from an ensemble workload's output: the rates
    of both sweep forms with their fractions of 8 TB/s, the speed-up over one
    launch per lattice and the mixed-vs-FP64 time to theta."""
    rate = lambda su, gbs: {"ms_per_launch": 1.0, "site_updates_per_s": su, "GBs": gbs}
    ens = {"configs": 48, "sites": 4860928, "sizes": [8, 12, 16, 24],
           "batched_fp32-12": rate(6.6e9, 5040.0), "batched_fp64-12": rate(3.3e9, 5080.0),
           "batched_fixed_fp32-12": rate(9.6e9, 5070.0), "batched_fixed_fp64-12": rate(4.8e9, 5010.0),
           "batched_speedup_fp32-12": 1.5,
           "gauge_fix_mixed_fixed_links": {"wall_s": 1.5}, "gauge_fix_fp64": {"wall_s": 4.05}}
    b = bench.batched_summary(ens)
    assert b["workload"].startswith("48 lattices of 8^4..24^4 (4860928 sites")
    for prefix, key in (("", "batched_"), ("fixed_", "batched_fixed_")):
        for name in ("fp32-12", "fp64-12"):
            assert b[f"{prefix}{name}_site_updates_per_s"] == ens[key + name]["site_updates_per_s"]
            assert b[f"{prefix}{name}_GBs"] == ens[key + name]["GBs"]
            assert b[f"{prefix}{name}_frac_of_8TBs"] == pytest.approx(ens[key + name]["GBs"] / 8000.0)
    assert b["speedup_vs_one_launch_per_lattice"] == 1.5
    assert b["time_to_theta_mixed_s"] == 1.5 and b["time_to_theta_fp64_s"] == 4.05
    assert b["mixed_speedup_vs_fp64"] == pytest.approx(2.7)
