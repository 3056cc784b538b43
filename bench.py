#!/usr/bin/env python3
"""Benchmark of the SU(3) Landau gauge-fixing hot path on one MI355X.

One step = one complete gauge fixing of the 64^4 workload (seeded synthetic
links: seed 3, eps 0.3, Haar-random gauge) from its stored start to
theta < 1e-14 with overrelaxation omega = 1.8, in the mixed form: FP32 12-real
bulk sweeps, FP64 reunitarization + F/theta every 20 sweeps, switch to FP64
(12-real storage) below theta = 1e-8, result handed back as FP64 18-real.  The
sweeps run in the fixed-link form (the links stay as stored, the sweeps update
the gauge transformation g and form g U g^dag in registers; the result is
g U g^dag from the input).  The start configuration stays resident in HBM (a
device-to-device copy opens each step).  value = site updates per second over
the whole step (V x sweeps / step time).

Also reported: the same gauge fixing with sweeps that rewrite the links, the
plain-FP64 time-to-theta on the same input, stochastic relaxation (p = 0.5)
sweep throughput, per-kernel roofline figures from HIP events, and the FP64 CPU
oracle timed on a bounded sample of the workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
# bytes per link as the sweeps read it (4: the split FP64 copy of the
# fixed-link form, FP32 rows plus 16-bit remainders) and per g(x) of the
# fixed-link form (4: FP64-12)
LINK_BYTES = {0: 144, 1: 72, 2: 48, 3: 96, 4: 72}
G_BYTES = {0: 144, 1: 72, 2: 48, 3: 96, 4: 96}


def fixed_site_bytes(fmt: int) -> int:
    """Algorithmic bytes per site update of the fixed-link sweep: 8 links in,
    g(x) in and out, and the neighbouring g of the other parity (each shared
    by the 8 sites around it) in once."""
    return 8 * LINK_BYTES[fmt] + 3 * G_BYTES[fmt]
# the sources that define the sweep kernels and their launch shape (the host
# driver only picks among them)
KERNEL_SOURCES = ["paper_1305_3440_amd/csrc/lgf_kernels.hip", "paper_1305_3440_amd/csrc/lgf_fixed.hip",
                  "paper_1305_3440_amd/csrc/lgf_device.hpp", "paper_1305_3440_amd/csrc/lgf_site.hpp",
                  "paper_1305_3440_amd/csrc/lgf_internal.hpp"]
# sweep variants the counter passes cover: (lanes per site, block, xcd remap, non-temporal, schedule)
TRAFFIC_VARIANTS = [(1, 128, 0, 1, 0), (2, 128, 0, 1, 0), (4, 128, 0, 1, 0), (1, 128, 0, 1, 2),
                    (2, 128, 0, 1, 2), (4, 128, 0, 1, 2), (1, 128, 0, 0, 0), (2, 128, 0, 0, 0)]
# fixed-link sweep variants the counter passes cover: (lanes per site, block, tile order)
TRAFFIC_FIXED_VARIANTS = [(lps, block, order) for lps in (2, 4) for block in (64, 128, 256) for order in (0, 1, 2)]
TRAFFIC_FIXED_SWEEPS = 4   # full sweeps per variant: 2 x 3 plain launches + the chunk's last sweep
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_64x4_hbm_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_key(fmt: int, lanes: int, nontemporal: int, schedule: int, dims) -> str:
    """Key of one sweep-kernel instance (format, lanes per site, non-temporal,
    out of place) on one lattice; the workgroup size does not change it."""
    return (f"sweep:fmt{fmt}:lanes{lanes}:nt{int(bool(nontemporal))}:oop{int(schedule == 2)}:"
            f"{'x'.join(map(str, dims))}")


def fixed_traffic_key(fmt: int, lanes: int, block: int, order: int, dims) -> str:
    """Key of one fixed-link sweep variant on one lattice (the tile order and
    the workgroup size set which neighbouring g come from the caches)."""
    return f"fixed:fmt{fmt}:lanes{lanes}:block{block}:order{order}:{'x'.join(map(str, dims))}"


def measured_traffic(key: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source and this kernel and workload."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != kernel_source_sha():
        return None
    e = t.get("kernels", {}).get(key)
    if not e:
        return None
    return e.get("hbm_bytes_per_launch")


def cpu_baseline(dims, seed, eps, omega, seconds):
    """The FP64 oracle on a 64^3 x 4 slab of the workload's shape (same
    generator and parameters), full OR sweeps for about `seconds`."""
    import oracle
    Lt = 4
    sdims = (Lt,) + tuple(dims[1:])
    U = oracle.generate_links(sdims, seed, eps, True)
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.sweep(sdims, U, omega, 0.0, 0, n)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or n >= 1000:
            break
    Vs = Lt * dims[1] * dims[2] * dims[3]
    # and the small 8^4 workload (seed 0, eps 0.25, Haar, omega 1.7) to theta < 1e-12
    d8 = (8, 8, 8, 8)
    U8 = oracle.generate_links(d8, 0, 0.25, True)
    t8 = time.perf_counter()
    r8 = oracle.gauge_fix(d8, U8, 1.7, 1e-12)
    t8 = time.perf_counter() - t8
    return {"value": Vs * n / el, "unit": "site-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{n} full OR sweeps (omega {omega}) of a {'x'.join(map(str, sdims))} slab "
                      f"({Vs} sites) with the 64^4 workload's generator (seed {seed}, eps {eps}, "
                      f"Haar), FP64, {el:.1f} s",
            "time_to_theta_8x4_s": t8, "sweeps_8x4": r8["sweeps"]}


def traffic_run(lgf, torch, dims, seed, eps, omega):
    """Workload for the rocprofv3 counter passes: a copy of known size (to
    calibrate FETCH_SIZE / WRITE_SIZE), then 4 sweep launches per format and
    sweep variant on the benchmark's 64^4 field."""
    n = 1 << 30
    a = torch.zeros(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    stream = torch.cuda.current_stream()
    for fmt in (lgf.LGF_FP32_12, lgf.LGF_FP64_12, lgf.LGF_FP64_18):
        h = lgf.lgf_create(dims, fmt, stream)
        lgf.lgf_generate_links(h, seed, eps, True)
        for v in TRAFFIC_VARIANTS:
            lgf.lgf_set_tuning(h, fmt, *v)
            ms = lgf.lgf_time_sweeps(h, 2, omega)
            log(f"[traffic] {lgf.FORMAT_NAMES[fmt]} {v}: {ms:.3f} ms per launch")
        lgf.lgf_destroy(h)
    # the fixed-link sweeps: TRAFFIC_FIXED_SWEEPS full sweeps per variant, in
    # the order of TRAFFIC_FIXED_VARIANTS (the summary groups the dispatches by it)
    h = lgf.lgf_create(dims, lgf.LGF_FP64_18, stream)
    lgf.lgf_generate_links(h, seed, eps, True)
    for fmt in (lgf.LGF_FP32_12, lgf.LGF_FP64_12, lgf.LGF_FP64_12S):
        for v in TRAFFIC_FIXED_VARIANTS:
            lgf.lgf_set_fixed_tuning(h, fmt, *v)
            p = lgf.fix_params(omega=omega, theta_target=1e-300, check_every=TRAFFIC_FIXED_SWEEPS,
                               max_sweeps=TRAFFIC_FIXED_SWEEPS, fixed_links=1, use_graph=0, bulk_format=fmt,
                               finish_format=fmt)
            st, res, _ = lgf.lgf_gauge_fix(h, p)
            log(f"[traffic] fixed {lgf.FORMAT_NAMES[fmt]} {v}: "
                f"{res['t_sweep_finish_ms'] / (2 * TRAFFIC_FIXED_SWEEPS):.3f} ms per launch")
    lgf.lgf_destroy(h)
    torch.cuda.synchronize()


def _find(dirpath, suffix):
    for root, _, files in os.walk(dirpath):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"no *{suffix} under {dirpath}")


def summarize_traffic(fetch_dir, write_dir, dims, command):
    import re
    """Per-launch HBM bytes of the sweep kernels from two rocprofv3 --pmc
    passes (FETCH_SIZE, WRITE_SIZE, KiB per dispatch), each scaled by the
    counter's reading for the 1 GiB copy; written next to the kernel-source
    hash so a stale figure is never reported."""
    import csv
    per = {}
    fixed_seq = {}  # (counter, format, lanes) -> plain fixed-sweep readings in dispatch order
    # fixed_sweep_kernel<format, lanes, SR, post, mu0>: the plain Landau instances
    fixed_pat = re.compile(r"fixed_sweep_kernel<(\d+),\s*(\d+),\s*false,\s*0,\s*0>")
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        with open(_find(d, "counter_collection.csv")) as f:
            rows = [r for r in csv.DictReader(f) if r.get("Counter_Name") == counter]
        rows.sort(key=lambda r: int(r.get("Dispatch_Id", 0)))
        for row in rows:
            per.setdefault((counter, row["Kernel_Name"]), []).append(float(row["Counter_Value"]))
            m = fixed_pat.search(row["Kernel_Name"])
            if m:
                fixed_seq.setdefault((counter, int(m.group(1)), int(m.group(2))), []).append(
                    float(row["Counter_Value"]))
    copy_bytes = float(1 << 30)
    out = {"source_sha": kernel_source_sha(), "command": command, "kernels": {}, "calibration": {}}
    scale = {}
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        vals = [v for (c, k), vs in per.items() if c == counter and "copyBuffer" in k for v in vs]
        kib = max(vals)  # the 1 GiB copy is the largest copy-kernel dispatch
        scale[counter] = copy_bytes / kib
        out["calibration"][counter] = {"copy_bytes": copy_bytes, "counter_kib": kib,
                                       "bytes_per_counter_unit": scale[counter]}
    # sweep_kernel<format, lanes per site, SR, non-temporal, out of place,
    # accumulate g, fused measurement>: the plain sweep instances
    pat = re.compile(r"sweep_kernel<(\d+),\s*(\d+),\s*(true|false),\s*(true|false),\s*(true|false),"
                     r"\s*false,\s*false>")
    Vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
    for (counter, kname), vals in per.items():
        m = pat.search(kname)
        if not m:
            continue
        fmt, lanes = int(m.group(1)), int(m.group(2))
        key = traffic_key(fmt, lanes, m.group(4) == "true", 2 if m.group(5) == "true" else 0, dims)
        e = out["kernels"].setdefault(key, {"kernel": kname, "format": fmt})
        e[counter.lower() + "_bytes_per_launch"] = sum(vals) / len(vals) * scale[counter]
        e[counter.lower() + "_dispatches"] = len(vals)
    # the fixed-link sweep: the plain (no reunitarization) launches of each
    # variant, 2 (TRAFFIC_FIXED_SWEEPS - 1) per variant, in the traffic run's order
    per_variant = 2 * (TRAFFIC_FIXED_SWEEPS - 1)
    for (counter, fmt, lanes), vals in fixed_seq.items():
        vs = [v for v in TRAFFIC_FIXED_VARIANTS if v[0] == lanes]
        for i, v in enumerate(vs):
            chunk = vals[i * per_variant:(i + 1) * per_variant]
            if len(chunk) != per_variant:
                continue
            key = fixed_traffic_key(fmt, v[0], v[1], v[2], dims)
            e = out["kernels"].setdefault(key, {"kernel": f"fixed_sweep_kernel<{fmt}, {lanes}, false, 0, 0>",
                                                "format": fmt, "fixed": True, "block": v[1], "order": v[2]})
            e[counter.lower() + "_bytes_per_launch"] = sum(chunk) / len(chunk) * scale[counter]
            e[counter.lower() + "_dispatches"] = len(chunk)
    for key, e in out["kernels"].items():
        # link sweep: 8 links in and out per site; fixed-link sweep: 8 links in,
        # g(x) in and out, the neighbouring g of the other parity in once
        alg = Vh * (fixed_site_bytes(e["format"]) if e.get("fixed") else 16 * LINK_BYTES[e["format"]])
        e["algorithmic_bytes_per_launch"] = alg
        e["hbm_bytes_per_launch"] = e.get("fetch_size_bytes_per_launch", 0) + e.get(
            "write_size_bytes_per_launch", 0)
        e["hbm_over_algorithmic"] = e["hbm_bytes_per_launch"] / alg
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def ensemble_bench(lgf, stream):
    """The 48-configuration batched workload (manifest under tests/golden):
    one persistent launch per parity over all lattices vs one launch per
    lattice, and the whole ensemble gauge-fixed (mixed) to theta < 1e-14."""
    man = json.load(open(os.path.join(ROOT, "tests", "golden", "ensemble48_manifest.json")))["configs"]
    dims = [tuple(c["dims"]) for c in man]
    Vtot = sum(d[0] * d[1] * d[2] * d[3] for d in dims)
    out = {"configs": len(dims), "sites": Vtot, "sizes": sorted({d[0] for d in dims})}
    e = lgf.lgf_ensemble_create(dims, lgf.LGF_FP64_18, stream)
    for c in man:
        lgf.lgf_ensemble_generate(e, c["index"], c["seed"], c["eps"], True)
    # tile width, persistent grid and non-temporal access picked on scratch copies
    lgf.lgf_ensemble_autotune(e, lgf.LGF_FP32_12, 2)
    out["tuning"] = dict(zip(("tile", "grid_mult", "nontemporal"), lgf.lgf_ensemble_get_tuning(e)))
    for fmt in (lgf.LGF_FP32_12, lgf.LGF_FP64_12):
        lgf.lgf_ensemble_time_sweeps(e, fmt, 20, 1.7)
        ms = lgf.lgf_ensemble_time_sweeps(e, fmt, 40, 1.7)
        by = Vtot // 2 * 16 * LINK_BYTES[fmt]
        out[f"batched_{lgf.FORMAT_NAMES[fmt]}"] = {"ms_per_launch": ms,
                                                   "site_updates_per_s": Vtot / 2 / (ms * 1e-3),
                                                   "GBs": by / (ms * 1e-3) / 1e9}
    # the same sweeps as one launch per lattice (each lattice its own handle)
    singles = []
    for c in man:
        h = lgf.lgf_create(tuple(c["dims"]), lgf.LGF_FP32_12, stream)
        lgf.lgf_generate_links(h, c["seed"], c["eps"], True)
        singles.append(h)
    for h in singles:
        lgf.lgf_time_sweeps(h, 2, 1.7)
    ms_loop = sum(lgf.lgf_time_sweeps(h, 10, 1.7) for h in singles)
    for h in singles:
        lgf.lgf_destroy(h)
    out["one_launch_per_lattice_fp32-12"] = {"ms_per_parity_sweep": ms_loop,
                                             "site_updates_per_s": Vtot / 2 / (ms_loop * 1e-3)}
    out["batched_speedup_fp32-12"] = ms_loop / out["batched_fp32-12"]["ms_per_launch"]
    p = lgf.lgf_fix_params_default()
    p.omega, p.theta_target, p.theta_switch = 1.7, 1e-14, 1e-8
    p.bulk_format, p.finish_format = lgf.LGF_FP32_12, lgf.LGF_FP64_12
    t0 = time.perf_counter()
    st, res = lgf.lgf_ensemble_gauge_fix(e, p, len(dims))
    wall = time.perf_counter() - t0
    # the same mixed gauge fixing with fixed-link sweeps (2 lanes per site)
    for c in man:
        lgf.lgf_ensemble_generate(e, c["index"], c["seed"], c["eps"], True)
    pf = lgf.fix_params(omega=1.7, theta_target=1e-14, theta_switch=1e-8, bulk_format=lgf.LGF_FP32_12,
                        finish_format=lgf.LGF_FP64_12, fixed_links=1)
    t0 = time.perf_counter()
    stf, resf = lgf.lgf_ensemble_gauge_fix(e, pf, len(dims))
    wallf = time.perf_counter() - t0
    # and with the FP64 finish on the split links
    for c in man:
        lgf.lgf_ensemble_generate(e, c["index"], c["seed"], c["eps"], True)
    ps = lgf.fix_params(omega=1.7, theta_target=1e-14, theta_switch=1e-8, bulk_format=lgf.LGF_FP32_12,
                        finish_format=lgf.LGF_FP64_12S, fixed_links=1)
    t0 = time.perf_counter()
    sts, ress = lgf.lgf_ensemble_gauge_fix(e, ps, len(dims))
    walls = time.perf_counter() - t0
    # the same 48 fields fixed in plain FP64 (18-real) for the per-configuration F difference
    for c in man:
        lgf.lgf_ensemble_generate(e, c["index"], c["seed"], c["eps"], True)
    p64 = lgf.lgf_fix_params_default()
    p64.omega, p64.theta_target = 1.7, 1e-14
    t0 = time.perf_counter()
    st64, res64 = lgf.lgf_ensemble_gauge_fix(e, p64, len(dims))
    wall64 = time.perf_counter() - t0
    lgf.lgf_ensemble_destroy(e)
    out["gauge_fix_fp64"] = {"status": int(st64), "wall_s": wall64,
                             "all_below_1e-14": all(r["theta"] < 1e-14 for r in res64)}
    out["max_abs_dF_mixed_vs_fp64"] = max(abs(r["F"] - q["F"]) for r, q in zip(res, res64))
    swf = [r["sweeps"] for r in resf]
    out["gauge_fix_mixed_fixed_links"] = {
        "status": int(stf), "wall_s": wallf, "all_below_1e-14": all(r["theta"] < 1e-14 for r in resf),
        "sweeps_min": min(swf), "sweeps_max": max(swf),
        "max_abs_dF_vs_fp64": max(abs(r["F"] - q["F"]) for r, q in zip(resf, res64)),
        "speedup_vs_link_sweeps": wall / wallf}
    sws = [r["sweeps"] for r in ress]
    out["gauge_fix_mixed_fixed_links_split_finish"] = {
        "status": int(sts), "wall_s": walls, "all_below_1e-14": all(r["theta"] < 1e-14 for r in ress),
        "sweeps_min": min(sws), "sweeps_max": max(sws),
        "max_abs_dF_vs_fp64": max(abs(r["F"] - q["F"]) for r, q in zip(ress, res64)),
        "max_abs_dF_vs_fp64_12_finish": max(abs(r["F"] - q["F"]) for r, q in zip(ress, resf)),
        "speedup_vs_fp64_12_finish": wallf / walls, "speedup_vs_link_sweeps": wall / walls}
    sw = [r["sweeps"] for r in res]
    out["gauge_fix_mixed"] = {"status": int(st), "wall_s": wall, "all_below_1e-14": all(
        r["theta"] < 1e-14 for r in res), "sweeps_min": min(sw), "sweeps_max": max(sw),
        "site_updates": sum(r["sweeps"] * d[0] * d[1] * d[2] * d[3] for r, d in zip(res, dims)),
        "site_updates_per_s": sum(r["sweeps"] * d[0] * d[1] * d[2] * d[3] for r, d in zip(res, dims)) / wall}
    return out


def gauge_32x4_bench(lgf, torch, stream):
    """32^4 (seed 1, eps 0.25, Haar, omega 1.7, theta < 1e-14): time-to-theta of
    plain FP64-18 and of the mixed runs (FP32-12 bulk, switch at 1e-8), and
    how far each run's plaquette moved from the input's.  The plaquette is
    gauge invariant, so an exact gauge transformation leaves it alone; the
    FP32 bulk without the accumulated transformation does not (the
    fixed-link sweeps keep the input links, so they stay on the orbit too)."""
    dims = (32, 32, 32, 32)
    dev = torch.device("cuda:0")
    home = lgf.LGF_FP64_18
    nbytes = lgf.lgf_required_bytes(dims, home)
    pristine = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    work = torch.empty_like(pristine)
    hp = lgf.lgf_create(dims, home, stream, pristine)
    lgf.lgf_generate_links(hp, 1, 0.25, True)
    hw = lgf.lgf_create(dims, home, stream, work)
    P0 = lgf.lgf_plaquette(hp)
    # (bulk, finish, accumulate_g, fixed_links)
    runs = {"fp64_18": (-1, -1, 0, 0), "mixed_fp32-12_to_fp64-18": (lgf.LGF_FP32_12, lgf.LGF_FP64_18, 0, 0),
            "mixed_fp32-12_to_fp64-12": (lgf.LGF_FP32_12, lgf.LGF_FP64_12, 0, 0),
            "mixed_fp32-12_to_fp64-12_accumulate_g": (lgf.LGF_FP32_12, lgf.LGF_FP64_12, 1, 0),
            "fp64_18_fixed_links": (-1, -1, 0, 1),
            "mixed_fp32-12_to_fp64-12_fixed_links": (lgf.LGF_FP32_12, lgf.LGF_FP64_12, 0, 1)}
    out = {"dims": list(dims), "plaquette_input": P0}
    for name, (bulk, finish, acc, fixed) in runs.items():
        p = lgf.lgf_fix_params_default()
        p.omega, p.theta_target, p.fixed_links = 1.7, 1e-14, fixed
        if bulk >= 0:
            p.theta_switch, p.bulk_format, p.finish_format, p.accumulate_g = 1e-8, bulk, finish, acc
        work.copy_(pristine)
        st, res, _ = lgf.lgf_gauge_fix(hw, p)
        out[name] = {"status": int(st), "time_to_theta_s": res["t_total_ms"] / 1e3, "sweeps": res["sweeps"],
                     "sweeps_bulk": res["sweeps_bulk"], "theta": res["theta"], "F": res["F"],
                     "plaquette_drift": lgf.lgf_plaquette(hw) - P0}
    for name in runs:
        if name != "fp64_18":
            out[name]["speedup_vs_fp64"] = out["fp64_18"]["time_to_theta_s"] / out[name]["time_to_theta_s"]
    lgf.lgf_destroy(hw)
    lgf.lgf_destroy(hp)
    del work, pristine
    torch.cuda.empty_cache()
    return out


def coulomb_bench(lgf, stream):
    """Coulomb gauge on 48^3 x 96 (seed 5, eps 0.3, Haar): the 96 timeslices
    relaxed together by one launch per parity, mixed FP32-12 bulk / FP64
    finish, omega 1.7, each timeslice stopping at its own theta_C < 1e-14: the
    fixed-link sweeps with the finish on the split links (reported first), on
    FP64-12 links, and the link-rewriting sweeps (FP64-12 finish)."""
    dims = (96, 48, 48, 48)
    V3 = dims[1] * dims[2] * dims[3]
    V = V3 * dims[0]
    h = lgf.lgf_create(dims, lgf.LGF_FP64_18, stream)

    def run(fixed, finish):
        # the same start for every run: the seeded generator, run again
        lgf.lgf_generate_links(h, 5, 0.3, True)
        p = lgf.fix_params(omega=1.7, theta_target=1e-14, theta_switch=1e-8, bulk_format=lgf.LGF_FP32_12,
                           finish_format=finish, fixed_links=fixed)
        lgf.lgf_synchronize(h)
        t0 = time.perf_counter()
        st, res, sw, F, th = lgf.lgf_coulomb_gauge_fix(h, p, dims[0])
        wall = time.perf_counter() - t0
        su = float(sw.sum()) * V3
        # algorithmic bytes per site update: link sweeps move 8 links in and
        # out; fixed-link sweeps read the 6 spatial links, g(x) in and out and
        # the neighbouring g once; FP32-12 bulk (every timeslice live), FP64
        # finish (live timeslices only)
        def per(fmt):
            return 6 * LINK_BYTES[fmt] + 3 * G_BYTES[fmt] if fixed else 16 * LINK_BYTES[fmt]
        su_bulk = float(res["sweeps_bulk"]) * V
        alg_bytes = su_bulk * per(lgf.LGF_FP32_12) + (su - su_bulk) * per(finish)
        t_sweep_s = (res["t_sweep_bulk_ms"] + res["t_sweep_finish_ms"]) / 1e3
        return {"status": int(st), "wall_s": wall, "sweeps_total": res["sweeps"],
                "sweep_algorithmic_GBs": alg_bytes / t_sweep_s / 1e9,
                "sweeps_bulk": res["sweeps_bulk"], "timeslice_sweeps_min": int(sw.min()),
                "timeslice_sweeps_max": int(sw.max()), "theta_max": float(th.max()), "F_mean": float(F.mean()),
                "site_updates": su, "site_updates_per_s": su / wall,
                "t_sweep_ms": res["t_sweep_bulk_ms"] + res["t_sweep_finish_ms"],
                "t_measure_ms": res["t_measure_ms"]}

    fixed = run(1, lgf.LGF_FP64_12S)
    fixed12 = run(1, lgf.LGF_FP64_12)
    link = run(0, lgf.LGF_FP64_12)
    lgf.lgf_destroy(h)
    out = {"dims": list(dims), "sweeps": "fixed-link, FP64 finish on split links", **fixed,
           "fixed_links_fp64_12_finish": fixed12, "link_sweeps": link,
           "fixed_speedup_vs_link_sweeps": link["wall_s"] / fixed["wall_s"],
           "split_speedup_vs_fp64_12_finish": fixed12["wall_s"] / fixed["wall_s"],
           "dF_mean_split_vs_fp64_12_finish": fixed["F_mean"] - fixed12["F_mean"]}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--dims", default="64,64,64,64")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP64 and SR reference runs")
    ap.add_argument("--traffic-run", action="store_true",
                    help="only the short workload of the rocprofv3 counter passes")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc output folders into profiles/sweep_64x4_hbm_traffic.json")
    ap.add_argument("--traffic-command", default="", help="command line recorded with the summary")
    ap.add_argument("--leg", choices=("coulomb", "ensemble", "gauge32"),
                    help="run only this extra workload and print its JSON (for profiling it alone)")
    args = ap.parse_args()
    if args.summarize_traffic:
        dims = tuple(int(x) for x in args.dims.split(","))
        summarize_traffic(args.summarize_traffic[0], args.summarize_traffic[1], dims,
                          args.traffic_command)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE {world}); the multi-GPU split is a design, not an implementation.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    sys.path.insert(0, ROOT)
    import paper_1305_3440_amd as lgf

    dims = tuple(int(x) for x in args.dims.split(","))
    V = dims[0] * dims[1] * dims[2] * dims[3]
    seed, eps, omega = 3, 0.3, 1.8
    theta_target, theta_switch = 1e-14, 1e-8
    # the finish reads the links from their split FP64 copy (FP64 arithmetic);
    # the link-rewriting comparison runs finish in FP64-12
    bulk, finish, home = lgf.LGF_FP32_12, lgf.LGF_FP64_12S, lgf.LGF_FP64_18
    finish12 = lgf.LGF_FP64_12
    stream = torch.cuda.current_stream()
    if args.traffic_run:
        traffic_run(lgf, torch, dims, seed, eps, omega)
        return
    if args.leg:
        legs = {"coulomb": lambda: coulomb_bench(lgf, stream), "ensemble": lambda: ensemble_bench(lgf, stream),
                "gauge32": lambda: gauge_32x4_bench(lgf, torch, stream)}
        print(json.dumps({"leg": args.leg, **legs[args.leg]()}), flush=True)
        return

    nbytes = lgf.lgf_required_bytes(dims, home)
    pristine = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    work = torch.empty_like(pristine)
    hp = lgf.lgf_create(dims, home, stream, pristine)
    lgf.lgf_generate_links(hp, seed, eps, True)
    hw = lgf.lgf_create(dims, home, stream, work)
    # sweep variants picked by the autotuners on this lattice: the fixed-link
    # sweeps of the step, and the link-rewriting sweeps of the comparison run
    lgf.lgf_autotune_fixed(hw, bulk, 4)
    lgf.lgf_autotune_fixed(hw, finish, 4)
    lgf.lgf_autotune(hw, bulk, 4)
    lgf.lgf_autotune(hw, finish12, 4)
    torch.cuda.synchronize()
    fixed_tuning = {f: lgf.lgf_get_fixed_tuning(hw, f) for f in (bulk, finish)}
    tuning = {f: lgf.lgf_get_tuning(hw, f) for f in (bulk, finish12, home)}
    log(f"[bench] {dims} V={V} generated; field {nbytes / 1e9:.2f} GB; fixed-link tuning (lanes, block, "
        f"order) fp32-12 {fixed_tuning[bulk]} fp64-12s {fixed_tuning[finish]}; link-sweep tuning fp32-12 "
        f"{tuning[bulk]} fp64-12 {tuning[finish12]}")

    params = lgf.lgf_fix_params_default()
    params.omega = omega
    params.theta_target = theta_target
    params.theta_switch = theta_switch
    params.bulk_format = bulk
    params.finish_format = finish
    params.check_every = 20
    params.use_graph = 1
    params.fixed_links = 1

    def step(p=params):
        work.copy_(pristine)
        st, res, hist = lgf.lgf_gauge_fix(hw, p)
        if st != lgf.LGF_OK:
            raise RuntimeError(f"gauge fix did not converge: {res}")
        return res

    for w in range(args.warmup):
        r = step()
        log(f"[bench] warmup {w}: {r['sweeps']} sweeps ({r['sweeps_bulk']} fp32-12), "
            f"theta {r['theta']:.3e}, {r['t_total_ms']:.0f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    total_sweeps = sum(r["sweeps"] for r in results)
    for i, r in enumerate(results):
        log(f"[bench] step {i}: {r['sweeps']} sweeps ({r['sweeps_bulk']} fp32-12), theta "
            f"{r['theta']:.3e}, F {r['F']:.12f}, {r['t_total_ms']:.0f} ms")

    # per-kernel figures from the driver's HIP events on the launch stream
    Vh = V // 2
    sb = sum(r["sweeps_bulk"] for r in results)
    sf = total_sweeps - sb
    tb = sum(r["t_sweep_bulk_ms"] for r in results)
    tf = sum(r["t_sweep_finish_ms"] for r in results)
    kernels = {}
    for name, fmt, nsw, tms in (("fixed_sweep_fp32_12", bulk, sb, tb), ("fixed_sweep_fp64_12s", finish, sf, tf)):
        if nsw > 0:
            launch_ms = tms / (2 * nsw)
            by = Vh * fixed_site_bytes(fmt)
            kernels[name] = {"launches": 2 * nsw, "avg_launch_ms": launch_ms,
                             "algorithmic_bytes_per_launch": by,
                             "achieved_GBs": by / (launch_ms * 1e-3) / 1e9,
                             "site_updates_per_s": Vh / (launch_ms * 1e-3), "total_ms": tms}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    dk = kernels[dom]
    dfmt = bulk if dom == "fixed_sweep_fp32_12" else finish
    fmt_name = lgf.FORMAT_NAMES[dfmt]
    lanes, block, order = fixed_tuning[dfmt]
    traffic = measured_traffic(fixed_traffic_key(dfmt, lanes, block, order, dims))
    roofline = {"bound": "hbm", "achieved": round(dk["achieved_GBs"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(dk["achieved_GBs"] / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "kernel": f"fixed_sweep_kernel<{fmt_name}, lanes/site {lanes}> block {block}, tile order "
                          f"{['lexicographic', 'XCD ranges', 't-z blocks per XCD'][order]}",
                "avg_launch_ms": round(dk["avg_launch_ms"], 4),
                "bytes_per_launch": dk["algorithmic_bytes_per_launch"]}

    if traffic:
        # the HBM bytes the counters saw per launch, at the launch time measured here
        roofline["traffic_GBs"] = round(traffic / (dk["avg_launch_ms"] * 1e-3) / 1e9, 1)
        roofline["traffic_frac"] = round(roofline["traffic_GBs"] / HBM_PEAK_GBS, 4)
    # the streaming ceiling on this GPU: a plain one-pass device copy of 4 GiB
    copy_gbs = lgf.lgf_copy_bandwidth(4 << 30, 10, stream)
    roofline["copy_ceiling_GBs"] = round(copy_gbs, 1)
    roofline["frac_of_copy_ceiling"] = round(dk["achieved_GBs"] / copy_gbs, 4)
    log(f"[bench] copy ceiling {copy_gbs:.1f} GB/s; dominant kernel at {dk['achieved_GBs']:.1f} GB/s")

    extras = {}
    if not args.no_extras:
        # the same mixed gauge fixing with sweeps that rewrite the links
        plink = lgf.fix_params(omega=omega, theta_target=theta_target, theta_switch=theta_switch,
                               bulk_format=bulk, finish_format=finish12, check_every=20, use_graph=1)
        rl = step(plink)
        extras["link_sweeps_mixed"] = {
            "time_to_theta_s": rl["t_total_ms"] / 1e3, "sweeps": rl["sweeps"], "sweeps_bulk": rl["sweeps_bulk"],
            "theta": rl["theta"], "F": rl["F"],
            "site_updates_per_s": V * rl["sweeps"] / (rl["t_total_ms"] / 1e3),
            "sweep_ms_per_launch": {"fp32-12": rl["t_sweep_bulk_ms"] / (2 * rl["sweeps_bulk"]),
                                    "fp64-12": rl["t_sweep_finish_ms"] / (2 * (rl["sweeps"] - rl["sweeps_bulk"]))},
            "tuning": {lgf.FORMAT_NAMES[f]: dict(zip(lgf.TUNING_FIELDS, tuning[f])) for f in (bulk, finish12)}}
        log(f"[bench] link sweeps, mixed: {rl['sweeps']} sweeps, {rl['t_total_ms']:.0f} ms, F {rl['F']:.12f}")
        # the same fixed-link gauge fixing with the finish on FP64-12 links
        lgf.lgf_autotune_fixed(hw, finish12, 4)
        p12 = lgf.fix_params(omega=omega, theta_target=theta_target, theta_switch=theta_switch,
                             bulk_format=bulk, finish_format=finish12, check_every=20, use_graph=1, fixed_links=1)
        r12 = step(p12)
        extras["fixed_links_fp64_12_finish"] = {
            "time_to_theta_s": r12["t_total_ms"] / 1e3, "sweeps": r12["sweeps"], "sweeps_bulk": r12["sweeps_bulk"],
            "theta": r12["theta"], "F": r12["F"],
            "site_updates_per_s": V * r12["sweeps"] / (r12["t_total_ms"] / 1e3),
            "fp64_12_ms_per_launch": r12["t_sweep_finish_ms"] / (2 * (r12["sweeps"] - r12["sweeps_bulk"])),
            "tuning": dict(zip(("lanes_per_site", "block", "order"), lgf.lgf_get_fixed_tuning(hw, finish12)))}
        log(f"[bench] fixed links, FP64-12 finish: {r12['sweeps']} sweeps, {r12['t_total_ms']:.0f} ms, "
            f"F {r12['F']:.15f}")
        # plain FP64 on the same input, its sweep variant autotuned the same way
        lgf.lgf_autotune(hw, home, 4)
        extras["fp64_plain_tuning"] = dict(zip(lgf.TUNING_FIELDS, lgf.lgf_get_tuning(hw, home)))
        p64 = lgf.lgf_fix_params_default()
        p64.omega = omega
        p64.theta_target = theta_target
        work.copy_(pristine)
        st, r64, _ = lgf.lgf_gauge_fix(hw, p64)
        extras["time_to_theta_fp64_s"] = r64["t_total_ms"] / 1e3
        extras["sweeps_fp64"] = r64["sweeps"]
        extras["F_fp64"] = r64["F"]
        extras["theta_fp64"] = r64["theta"]
        launch64 = r64["t_sweep_finish_ms"] / (2 * r64["sweeps"])
        extras["fp64_plain_sweep_GBs"] = Vh * 2304 / (launch64 * 1e-3) / 1e9
        # stochastic relaxation p = 0.5 (omega 1), Philox keyed by (site, sweep)
        work.copy_(pristine)
        ms_sr64 = lgf.lgf_time_sweeps(hw, 10, 1.0, 0.5, 17, 0)
        hsr = lgf.lgf_create(dims, bulk, stream)
        lgf.lgf_generate_links(hsr, seed, eps, True)
        ms_sr32 = lgf.lgf_time_sweeps(hsr, 10, 1.0, 0.5, 17, 0)
        ms_or32 = lgf.lgf_time_sweeps(hsr, 10, omega, 0.0, 0, 0)
        lgf.lgf_destroy(hsr)
        extras["sr_p0.5_fp64_18"] = {"site_updates_per_s": Vh / (ms_sr64 * 1e-3),
                                     "GBs": Vh * 2304 / (ms_sr64 * 1e-3) / 1e9}
        extras["sr_p0.5_fp32_12"] = {"site_updates_per_s": Vh / (ms_sr32 * 1e-3),
                                     "GBs": Vh * 768 / (ms_sr32 * 1e-3) / 1e9}
        extras["or_fp32_12_isolated"] = {"site_updates_per_s": Vh / (ms_or32 * 1e-3),
                                         "GBs": Vh * 768 / (ms_or32 * 1e-3) / 1e9}
        mixed_s = sum(r["t_total_ms"] for r in results) / len(results) / 1e3
        extras["time_to_theta_mixed_s"] = mixed_s
        extras["mixed_speedup_vs_fp64"] = extras["time_to_theta_fp64_s"] / mixed_s
        extras["dF_mixed_vs_fp64"] = results[-1]["F"] - r64["F"]
        extras["dF_link_sweeps_mixed_vs_fp64"] = rl["F"] - r64["F"]
        extras["fixed_speedup_vs_link_sweeps"] = extras["link_sweeps_mixed"]["time_to_theta_s"] / mixed_s
        extras["split_speedup_vs_fp64_12_finish"] = extras["fixed_links_fp64_12_finish"]["time_to_theta_s"] / mixed_s
        extras["dF_split_vs_fp64_12_finish"] = results[-1]["F"] - r12["F"]
        log(f"[bench] fp64 plain: {r64['sweeps']} sweeps, {r64['t_total_ms']:.0f} ms; "
            f"SR fp64 {ms_sr64:.3f} ms/launch, SR fp32-12 {ms_sr32:.3f}, OR fp32-12 {ms_or32:.3f}")
    lgf.lgf_destroy(hw)
    lgf.lgf_destroy(hp)
    del work, pristine
    torch.cuda.empty_cache()
    if not args.no_extras:
        # the small 8^4 workload to theta < 1e-12, plain FP64-18 (its oracle time is in cpu_baseline)
        h8 = lgf.lgf_create((8, 8, 8, 8), home, stream)
        lgf.lgf_generate_links(h8, 0, 0.25, True)
        p8 = lgf.lgf_fix_params_default()
        p8.omega, p8.theta_target = 1.7, 1e-12
        lgf.lgf_synchronize(h8)
        st8, r8, _ = lgf.lgf_gauge_fix(h8, p8)
        lgf.lgf_destroy(h8)
        extras["gauge_8x4"] = {"status": int(st8), "sweeps": r8["sweeps"],
                               "time_to_theta_s": r8["t_total_ms"] / 1e3, "theta": r8["theta"]}
        log("[bench] 32^4 plain vs mixed, plaquette drift")
        extras["gauge_32x4"] = gauge_32x4_bench(lgf, torch, stream)
        log(f"[bench] 32^4: {json.dumps(extras['gauge_32x4'])}")
        log("[bench] 48-configuration ensemble")
        extras["ensemble48"] = ensemble_bench(lgf, stream)
        log(f"[bench] ensemble: {json.dumps(extras['ensemble48'])}")
        log("[bench] Coulomb gauge 48^3 x 96")
        extras["coulomb_48x3x96"] = coulomb_bench(lgf, stream)
        log(f"[bench] coulomb: {json.dumps(extras['coulomb_48x3x96'])}")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host")
        cpu = cpu_baseline(dims, seed, eps, omega, args.cpu_seconds)

    out = {
        "metric": "OR site-updates/s (64^4 Landau gauge fixing to theta<1e-14, mixed FP32-12/FP64)",
        "value": V * total_sweeps / elapsed,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32+fp64",
        "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, dims))} SU(3) Landau OR gauge fixing, mixed "
                               f"FP32-12 bulk / FP64 finish (FP64 arithmetic and g; links read from a split "
                               f"copy, fl32 + 16-bit remainder, within 2^-40), theta<1e-14 measured on the "
                               f"FP64 result, fixed-link sweeps",
                   "dims": list(dims), "seed": seed, "eps": eps, "haar": True, "omega": omega,
                   "theta_target": theta_target, "theta_switch": theta_switch, "check_every": 20,
                   "sweeps_per_step": [r["sweeps"] for r in results],
                   "fixed_sweep_tuning": {lgf.FORMAT_NAMES[f]: dict(zip(("lanes_per_site", "block", "order"), t))
                                          for f, t in fixed_tuning.items()}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "step_breakdown_ms": {k: sum(r[k] for r in results) / len(results)
                              for k in ("t_sweep_bulk_ms", "t_sweep_finish_ms", "t_measure_ms", "t_convert_ms",
                                        "t_total_ms")},
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
