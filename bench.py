#!/usr/bin/env python3
"""Benchmark of the SU(3) Landau gauge-fixing hot path on one MI355X.

Workload: the 64^4 lattice of seeded synthetic links (seed 3, eps 0.3, then a
Haar-random gauge transformation), overrelaxation omega = 1.8.

One step = one check interval of the FP64 gauge fixing on that lattice: 20
full sweeps (parity 0, then parity 1) of the fixed-link form replayed from a
hipGraph, the gauge transformation reunitarized in FP64 as the last sweep
stores it, and F, theta measured in FP64 (Sec. 4: sweep the parities in turn,
check theta).  The sweeps compute in FP64 on links and gauge transformation
stored in FP64 12-real form (rows 0 and 1; row 2 rebuilt).  The field and the
gauge transformation stay resident in HBM between steps; a step is the unit
the gauge fixing repeats until theta < 1e-14.  value = site updates per
second (V x 20 x steps / timed wall time).

Reported beside it, each run once: time to theta < 1e-14 of the mixed form
(FP32 12-real bulk, FP64 finish below theta = 1e-8, and again below 1e-11) and
of the plain FP64 form on the same input, the same with the finish reading the links from a split
copy (fl32 + 16-bit remainder), the paper's link-rewriting FP64 form, the
roofline of the dominant kernel from HIP events, the FP64 CPU oracle timed
on 10 sweeps of the same 64^4 field on all host cores and on one more sweep
on one core, the batched form (48 lattices of 8^4..24^4 in one persistent
launch per parity) against one launch per lattice and against plain FP64, and
the overrelaxation kernels at 32^4 per storage format.
Optional items are skipped (and say so) past a wall-clock budget.  Other
workloads run alone through --leg (link64, gauge32, ensemble, coulomb, anneal,
or32, switch).

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--budget 460]
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
# fixed-link sweep variants the counter passes cover, per sweep format:
# (lanes per site, block, tile order, link layout)
TRAFFIC_FIXED_VARIANTS = {
    2: [(lps, block, order, layout) for lps in (1, 2) for block in (64, 128, 256) for order in (0, 3)
        for layout in (0, 1)],
    3: [(2, block, order, layout) for block in (64, 128, 256) for order in (0, 2, 3) for layout in (0, 1)] +
       [(4, 256, order, layout) for order in (2, 3) for layout in (0, 1)],
    4: [(2, block, order, layout) for block in (64, 128, 256) for order in (0, 2, 3) for layout in (0, 1)],
}
FIXED_TUNING_KEYS = ("lanes_per_site", "block", "order", "layout")
LOW_SWITCH = 1e-11   # a later precision switch of the mixed form, reported beside the 1e-8 one
TILE_ORDERS = ["lexicographic", "XCD ranges", "t-z blocks per XCD", "lockstep planes, an eighth per XCD"]
LINK_LAYOUTS = ["link field", "per-site link records"]
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


def fixed_traffic_key(fmt: int, lanes: int, block: int, order: int, layout: int, dims) -> str:
    """Key of one fixed-link sweep variant on one lattice (the tile order and
    the workgroup size set which neighbouring g come from the caches)."""
    return f"fixed:fmt{fmt}:lanes{lanes}:block{block}:order{order}:layout{layout}:{'x'.join(map(str, dims))}"


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


def cpu_baseline(dims, seed, eps, omega, sweeps, max_seconds):
    """The FP64 oracle on the host cores: full OR sweeps of the benchmark's own
    field (the same generator and parameters, generated on the host, not
    timed), `sweeps` of them or as many as fit in `max_seconds`; and the 8^4
    workload (seed 0, eps 0.25, Haar, omega 1.7) to theta < 1e-12."""
    import oracle
    t_gen = time.perf_counter()
    U = oracle.generate_links(dims, seed, eps, True)
    t_gen = time.perf_counter() - t_gen
    n = 0
    t0 = time.perf_counter()
    while n < sweeps:
        oracle.sweep(dims, U, omega, 0.0, 0, n)
        n += 1
        if time.perf_counter() - t0 >= max_seconds:
            break
    el = time.perf_counter() - t0
    cores = oracle.num_threads()
    # the same oracle on one core: one more full sweep of the same field
    oracle.set_num_threads(1)
    t1 = time.perf_counter()
    oracle.sweep(dims, U, omega, 0.0, 0, n)
    el1 = time.perf_counter() - t1
    oracle.set_num_threads(cores)
    del U
    V = dims[0] * dims[1] * dims[2] * dims[3]
    d8 = (8, 8, 8, 8)
    U8 = oracle.generate_links(d8, 0, 0.25, True)
    t8 = time.perf_counter()
    r8 = oracle.gauge_fix(d8, U8, 1.7, 1e-12)
    t8 = time.perf_counter() - t8
    return {"value": V * n / el, "unit": "site-updates/s", "cores": cores,
            "kind": "oracle",
            "single_thread": {"value": V / el1, "unit": "site-updates/s", "cores": 1,
                              "sample": f"1 full OR sweep of the same field, {el1:.1f} s"},
            "sample": f"{n} full OR sweeps (omega {omega}) of the {'x'.join(map(str, dims))} workload's field "
                      f"(seed {seed}, eps {eps}, Haar; generated on the host in {t_gen:.1f} s, not timed), "
                      f"FP64, {el:.1f} s",
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
        for v in TRAFFIC_FIXED_VARIANTS[fmt]:
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
    fixed_seq = {}  # (counter, format, lanes, layout) -> plain fixed-sweep readings in dispatch order
    # fixed_sweep_kernel<format, lanes, SR, post, mu0, records>: the plain Landau instances
    fixed_pat = re.compile(r"fixed_sweep_kernel<(\d+),\s*(\d+),\s*false,\s*0,\s*0,\s*(true|false)>")
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        with open(_find(d, "counter_collection.csv")) as f:
            rows = [r for r in csv.DictReader(f) if r.get("Counter_Name") == counter]
        rows.sort(key=lambda r: int(r.get("Dispatch_Id", 0)))
        for row in rows:
            per.setdefault((counter, row["Kernel_Name"]), []).append(float(row["Counter_Value"]))
            m = fixed_pat.search(row["Kernel_Name"])
            if m:
                fixed_seq.setdefault((counter, int(m.group(1)), int(m.group(2)), int(m.group(3) == "true")),
                                     []).append(float(row["Counter_Value"]))
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
    for (counter, fmt, lanes, layout), vals in fixed_seq.items():
        vs = [v for v in TRAFFIC_FIXED_VARIANTS.get(fmt, []) if v[0] == lanes and v[3] == layout]
        for i, v in enumerate(vs):
            chunk = vals[i * per_variant:(i + 1) * per_variant]
            if len(chunk) != per_variant:
                continue
            key = fixed_traffic_key(fmt, v[0], v[1], v[2], v[3], dims)
            e = out["kernels"].setdefault(key, {"kernel": f"fixed_sweep_kernel<{fmt}, {lanes}, false, 0, 0, "
                                                          f"{'true' if layout else 'false'}>",
                                                "format": fmt, "fixed": True, "block": v[1], "order": v[2],
                                                "layout": v[3]})
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


def mixed_bulk_summary(fmt, tuning, Vh, bulk_ms, fp64_launch_ms):
    """The mixed form's bulk sweep (format fmt, its fixed-link tuning (lanes
    per site, block, tile order, link layout)) at ms per launch over Vh site
    updates, against the FP64 sweep of the step at fp64_launch_ms."""
    lanes, block, order, layout = tuning
    gbs = Vh * fixed_site_bytes(fmt) / (bulk_ms * 1e-3) / 1e9
    return {"kernel": f"fixed_sweep_kernel<fp32-12, lanes/site {lanes}> block {block}, tile order "
                      f"{TILE_ORDERS[order]}, links from the {LINK_LAYOUTS[layout]}",
            "ms_per_launch": round(bulk_ms, 4), "site_updates_per_s": Vh / (bulk_ms * 1e-3),
            "GBs": round(gbs, 1), "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_per_site_update": fixed_site_bytes(fmt),
            "site_updates_vs_fp64_sweep": round(fp64_launch_ms / bulk_ms, 3)}


def batched_summary(ens):
    """The line's `batched` object from the ensemble workload's output
    (ensemble_bench): the persistent launches' rates in both sweep forms with
    their fraction of 8 TB/s, the speed-up over one launch per lattice, and
    the ensemble's time to theta mixed (fixed-link form) against plain FP64."""
    out = {"workload": f"{ens['configs']} lattices of {min(ens['sizes'])}^4..{max(ens['sizes'])}^4 "
                       f"({ens['sites']} sites, seeds 100..147), one persistent launch per parity"}
    for prefix, key in (("", "batched_"), ("fixed_", "batched_fixed_")):
        for name in ("fp32-12", "fp64-12"):
            r = ens[key + name]
            out[f"{prefix}{name}_site_updates_per_s"] = r["site_updates_per_s"]
            out[f"{prefix}{name}_GBs"] = r["GBs"]
            out[f"{prefix}{name}_frac_of_8TBs"] = r["GBs"] / HBM_PEAK_GBS
    mixed_e, plain_e = ens["gauge_fix_mixed_fixed_links"]["wall_s"], ens["gauge_fix_fp64"]["wall_s"]
    out.update({"speedup_vs_one_launch_per_lattice": ens["batched_speedup_fp32-12"],
                "time_to_theta_mixed_s": mixed_e, "time_to_theta_fp64_s": plain_e,
                "mixed_speedup_vs_fp64": plain_e / mixed_e})
    return out


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
    # the fixed-link form of the same launches (the mixed fixing below runs
    # it): the links read from their per-site records, g(x) read and written
    for fmt in (lgf.LGF_FP32_12, lgf.LGF_FP64_12):
        lgf.lgf_ensemble_time_fixed_sweeps(e, fmt, 20, 1.7)
        ms = lgf.lgf_ensemble_time_fixed_sweeps(e, fmt, 40, 1.7)
        by = Vtot // 2 * fixed_site_bytes(fmt)
        out[f"batched_fixed_{lgf.FORMAT_NAMES[fmt]}"] = {"ms_per_launch": ms,
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


def link64_bench(lgf, torch, stream, dims, seed, eps, omega):
    """The 64^4 workload's other forms, each timed once: the mixed gauge fixing
    with sweeps that rewrite the links (autotuned variants), the fixed-link
    one with its finish on FP64-12 links instead of the split copy, and the
    sweep rates of stochastic relaxation (p = 0.5, Philox keyed by site and
    sweep) and of overrelaxation in FP32-12 and FP64-18."""
    dev = torch.device("cuda:0")
    V = dims[0] * dims[1] * dims[2] * dims[3]
    Vh = V // 2
    bulk, home, finish12 = lgf.LGF_FP32_12, lgf.LGF_FP64_18, lgf.LGF_FP64_12
    nbytes = lgf.lgf_required_bytes(dims, home)
    pristine = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    work = torch.empty_like(pristine)
    hp = lgf.lgf_create(dims, home, stream, pristine)
    lgf.lgf_generate_links(hp, seed, eps, True)
    hw = lgf.lgf_create(dims, home, stream, work)
    out = {"dims": list(dims)}
    lgf.lgf_autotune(hw, bulk, 4)
    lgf.lgf_autotune(hw, finish12, 4)
    plink = lgf.fix_params(omega=omega, theta_target=1e-14, theta_switch=1e-8, bulk_format=bulk,
                           finish_format=finish12)
    work.copy_(pristine)
    st, rl, _ = lgf.lgf_gauge_fix(hw, plink)
    out["link_sweeps_mixed"] = {
        "status": int(st), "time_to_theta_s": rl["t_total_ms"] / 1e3, "sweeps": rl["sweeps"],
        "sweeps_bulk": rl["sweeps_bulk"], "theta": rl["theta"], "F": rl["F"],
        "sweep_ms_per_launch": {"fp32-12": rl["t_sweep_bulk_ms"] / (2 * max(rl["sweeps_bulk"], 1)),
                                "fp64-12": rl["t_sweep_finish_ms"] / (2 * max(rl["sweeps"] - rl["sweeps_bulk"], 1))},
        "tuning": {lgf.FORMAT_NAMES[f]: dict(zip(lgf.TUNING_FIELDS, lgf.lgf_get_tuning(hw, f)))
                   for f in (bulk, finish12)}}
    log(f"[link64] link sweeps, mixed: {json.dumps(out['link_sweeps_mixed'])}")
    p12 = lgf.fix_params(omega=omega, theta_target=1e-14, theta_switch=1e-8, bulk_format=bulk,
                         finish_format=finish12, fixed_links=1)
    work.copy_(pristine)
    st, r12, _ = lgf.lgf_gauge_fix(hw, p12)
    out["fixed_links_fp64_12_finish"] = {
        "status": int(st), "time_to_theta_s": r12["t_total_ms"] / 1e3, "sweeps": r12["sweeps"],
        "sweeps_bulk": r12["sweeps_bulk"], "theta": r12["theta"], "F": r12["F"],
        "fp64_12_ms_per_launch": r12["t_sweep_finish_ms"] / (2 * max(r12["sweeps"] - r12["sweeps_bulk"], 1))}
    log(f"[link64] fixed links, FP64-12 finish: {json.dumps(out['fixed_links_fp64_12_finish'])}")
    work.copy_(pristine)
    ms_sr64 = lgf.lgf_time_sweeps(hw, 10, 1.0, 0.5, 17, 0)
    ms_or64 = lgf.lgf_time_sweeps(hw, 10, omega, 0.0, 0, 0)
    hsr = lgf.lgf_create(dims, bulk, stream)
    lgf.lgf_generate_links(hsr, seed, eps, True)
    ms_sr32 = lgf.lgf_time_sweeps(hsr, 10, 1.0, 0.5, 17, 0)
    ms_or32 = lgf.lgf_time_sweeps(hsr, 10, omega, 0.0, 0, 0)
    lgf.lgf_destroy(hsr)
    for name, ms, by in (("sr_p0.5_fp64_18", ms_sr64, 2304), ("or_fp64_18", ms_or64, 2304),
                         ("sr_p0.5_fp32_12", ms_sr32, 768), ("or_fp32_12", ms_or32, 768)):
        out[name] = {"ms_per_launch": ms, "site_updates_per_s": Vh / (ms * 1e-3),
                     "GBs": Vh * by / (ms * 1e-3) / 1e9}
    lgf.lgf_destroy(hw)
    lgf.lgf_destroy(hp)
    del work, pristine
    torch.cuda.empty_cache()
    return out


def switch_bench(lgf, torch, stream, dims, seed, eps, omega, switches):
    """Where the mixed gauge fixing of the 64^4 workload (fixed-link form,
    FP32-12 bulk, FP64-12 finish, autotuned) leaves FP32: time to theta <
    1e-14 for each switch precision (the first is the reference), each once
    from the same input, with F against the first run.  A bulk that cannot
    reach its switch stops at max_sweeps (status LGF_ENOTCONV)."""
    dev = torch.device("cuda:0")
    bulk, home, finish = lgf.LGF_FP32_12, lgf.LGF_FP64_18, lgf.LGF_FP64_12
    nbytes = lgf.lgf_required_bytes(dims, home)
    pristine = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    work = torch.empty_like(pristine)
    hp = lgf.lgf_create(dims, home, stream, pristine)
    lgf.lgf_generate_links(hp, seed, eps, True)
    hw = lgf.lgf_create(dims, home, stream, work)
    work.copy_(pristine)
    lgf.lgf_autotune_fixed(hw, finish, 4)
    lgf.lgf_autotune_fixed(hw, bulk, 4)
    out = {"dims": list(dims), "fixed_sweep_tuning": {lgf.FORMAT_NAMES[f]: dict(zip(FIXED_TUNING_KEYS,
                                                                                   lgf.lgf_get_fixed_tuning(hw, f)))
                                                      for f in (bulk, finish)}}
    F_ref = None
    for sw in switches:
        p = lgf.fix_params(omega=omega, theta_target=1e-14, theta_switch=sw, bulk_format=bulk,
                           finish_format=finish, fixed_links=1, max_sweeps=30000)
        work.copy_(pristine)
        st, r, _ = lgf.lgf_gauge_fix(hw, p)
        e = {"status": lgf.STATUS_NAMES.get(int(st), int(st)), "time_to_theta_s": r["t_total_ms"] / 1e3,
             "sweeps": r["sweeps"], "sweeps_bulk": r["sweeps_bulk"], "theta": r["theta"], "F": r["F"],
             "t_sweep_bulk_s": r["t_sweep_bulk_ms"] / 1e3, "t_sweep_finish_s": r["t_sweep_finish_ms"] / 1e3}
        if F_ref is None:
            F_ref = r["F"]
        e["dF_vs_first"] = r["F"] - F_ref
        out[f"switch_{sw:.0e}"] = e
        log(f"[switch] {sw:.0e}: {json.dumps(e)}")
    lgf.lgf_destroy(hw)
    lgf.lgf_destroy(hp)
    del work, pristine
    torch.cuda.empty_cache()
    return out


def or_kernels_32x4(lgf, stream, omega):
    """The paper's single-GPU measurement (Sec. 4, Fig. 1: the overrelaxation
    kernel on a 32^4 lattice in single, mixed and double precision), per
    storage format: site updates per second of one launch (a half-sweep) of
    the link-rewriting sweep (autotuned) and of the fixed-link sweep
    (its autotuned variant, inside a stepwise session), with the launch's
    algorithmic bytes.  The 32^4 field (seed 1, eps 0.25, Haar gauge) is
    generated on the device."""
    dims = (32, 32, 32, 32)
    Vh = 32 ** 4 // 2
    out = {"dims": list(dims)}
    for fmt in (lgf.LGF_FP32_12, lgf.LGF_FP32_18, lgf.LGF_FP64_12, lgf.LGF_FP64_18):
        h = lgf.lgf_create(dims, fmt, stream)
        lgf.lgf_generate_links(h, 1, 0.25, True)
        lgf.lgf_autotune(h, fmt, 4)
        lgf.lgf_time_sweeps(h, 20, omega)
        ms = lgf.lgf_time_sweeps(h, 100, omega)
        lgf.lgf_destroy(h)
        out[f"link_sweep_{lgf.FORMAT_NAMES[fmt]}"] = {
            "ms_per_launch": ms, "site_updates_per_s": Vh / (ms * 1e-3),
            "GBs": Vh * 16 * LINK_BYTES[fmt] / (ms * 1e-3) / 1e9}
    h = lgf.lgf_create(dims, lgf.LGF_FP64_18, stream)
    lgf.lgf_generate_links(h, 1, 0.25, True)
    for fmt in (lgf.LGF_FP32_12, lgf.LGF_FP64_12):
        lgf.lgf_autotune_fixed(h, fmt, 4)
        lgf.lgf_fix_begin(h, fmt)
        lgf.lgf_fix_chunk(h, 20, omega)
        ms = sum(lgf.lgf_fix_chunk(h, 20, omega, 0.0, 0, 20 * (k + 1))[2] for k in range(5)) / (5 * 40)
        lgf.lgf_fix_end(h)
        out[f"fixed_sweep_{lgf.FORMAT_NAMES[fmt]}"] = {
            "ms_per_launch": ms, "site_updates_per_s": Vh / (ms * 1e-3),
            "GBs": Vh * fixed_site_bytes(fmt) / (ms * 1e-3) / 1e9}
    lgf.lgf_destroy(h)
    return out


def anneal_bench(lgf, torch, stream, dims, seed, eps, omega):
    """Simulated annealing on the 64^4 workload (FP64-12 handle, link-
    rewriting heat-bath sweeps): the sweep rate of a 100-sweep schedule
    (T 1.0 -> 0.05) with its algorithmic bytes (8 links read and written per
    site update), then overrelaxation (fixed-link mixed form) to theta < 1e-14,
    against the same overrelaxation without annealing: time, sweeps and the
    F reached (annealing is meant to reach a higher maximum)."""
    V = dims[0] * dims[1] * dims[2] * dims[3]
    fmt = lgf.LGF_FP64_12
    h = lgf.lgf_create(dims, fmt, stream)
    out = {"dims": list(dims), "format": lgf.FORMAT_NAMES[fmt], "schedule": {"sweeps": 100, "T_start": 1.0,
                                                                             "T_end": 0.05}}

    def fix():
        p = lgf.fix_params(omega=omega, theta_target=1e-14, theta_switch=1e-8, bulk_format=lgf.LGF_FP32_12,
                           finish_format=lgf.LGF_FP64_12, fixed_links=1)
        st, r, _ = lgf.lgf_gauge_fix(h, p)
        return {"status": lgf.STATUS_NAMES.get(int(st), int(st)), "time_s": r["t_total_ms"] / 1e3,
                "sweeps": r["sweeps"], "F": r["F"], "theta": r["theta"]}

    lgf.lgf_generate_links(h, seed, eps, True)
    out["overrelaxation_only"] = fix()
    log(f"[anneal] overrelaxation only: {json.dumps(out['overrelaxation_only'])}")
    lgf.lgf_generate_links(h, seed, eps, True)
    lgf.lgf_anneal(h, 4, 1.0, 1.0, 99, 1000)  # warm-up of the kernel
    lgf.lgf_generate_links(h, seed, eps, True)
    lgf.lgf_synchronize(h)
    trials, ms = lgf.lgf_anneal(h, 100, 1.0, 0.05, 7, 0)
    # 100 sweeps moving 8 links in and out per site update (FP64-12: 1536 B),
    # 5 reunitarizations reading and writing every link (768 B per site)
    by = 100 * V * 1536 + 5 * V * 768
    out["anneal"] = {"ms": ms, "trials_per_subgroup_step": trials / (3 * V * 100),
                     "site_updates_per_s": V * 100 / (ms * 1e-3), "algorithmic_GBs": by / (ms * 1e-3) / 1e9,
                     "frac_of_8TBs": by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    F0, th0 = lgf.lgf_measure(h)
    out["anneal"]["F_after"], out["anneal"]["theta_after"] = F0, th0
    log(f"[anneal] schedule: {json.dumps(out['anneal'])}")
    out["anneal_then_overrelaxation"] = fix()
    out["dF_anneal_vs_overrelaxation_only"] = out["anneal_then_overrelaxation"]["F"] - out["overrelaxation_only"]["F"]
    lgf.lgf_destroy(h)
    return out


def main():
    t_begin = time.perf_counter()
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dims", default="64,64,64,64")
    ap.add_argument("--budget", type=float, default=460.0,
                    help="wall-clock seconds after which optional items are skipped")
    ap.add_argument("--cpu-sweeps", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed steps and the roofline (no time-to-theta runs)")
    ap.add_argument("--traffic-run", action="store_true",
                    help="only the short workload of the rocprofv3 counter passes")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc output folders into profiles/sweep_64x4_hbm_traffic.json")
    ap.add_argument("--traffic-command", default="", help="command line recorded with the summary")
    ap.add_argument("--leg", choices=("coulomb", "ensemble", "gauge32", "link64", "anneal", "or32", "switch"),
                    help="run only this extra workload and print its JSON")
    ap.add_argument("--switches", default="1e-8,1e-9,1e-10,1e-11",
                    help="switch precisions of --leg switch (comma separated)")
    args = ap.parse_args()
    if args.summarize_traffic:
        dims = tuple(int(x) for x in args.dims.split(","))
        summarize_traffic(args.summarize_traffic[0], args.summarize_traffic[1], dims,
                          args.traffic_command)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this implementation runs on one GPU only (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE {world}); the multi-GPU split is a design, not an implementation.",
              file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("bench.py: --steps must be >= 1 and --warmup >= 0", file=sys.stderr)
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
    Vh = V // 2
    seed, eps, omega = 3, 0.3, 1.8
    theta_target, theta_switch = 1e-14, 1e-8
    chunk = 20
    # the step's sweeps: FP64 arithmetic on FP64-12 links and g; the mixed
    # form's bulk in FP32-12; the handle's links in FP64-18; the split copy of
    # the links (FP64 arithmetic, links within 2^-40) as an extra finish
    finish, bulk, home, split = lgf.LGF_FP64_12, lgf.LGF_FP32_12, lgf.LGF_FP64_18, lgf.LGF_FP64_12S
    stream = torch.cuda.current_stream()
    if args.traffic_run:
        traffic_run(lgf, torch, dims, seed, eps, omega)
        return
    if args.leg:
        legs = {"coulomb": lambda: coulomb_bench(lgf, stream), "ensemble": lambda: ensemble_bench(lgf, stream),
                "gauge32": lambda: gauge_32x4_bench(lgf, torch, stream),
                "link64": lambda: link64_bench(lgf, torch, stream, dims, seed, eps, omega),
                "anneal": lambda: anneal_bench(lgf, torch, stream, dims, seed, eps, omega),
                "or32": lambda: or_kernels_32x4(lgf, stream, 1.7),
                "switch": lambda: switch_bench(lgf, torch, stream, dims, seed, eps, omega,
                                               [float(x) for x in args.switches.split(",")])}
        print(json.dumps({"leg": args.leg, **legs[args.leg]()}), flush=True)
        return

    def elapsed():
        return time.perf_counter() - t_begin

    skipped = []

    def fits(name, seconds):
        """Whether an optional item of about `seconds` still fits the budget."""
        if elapsed() + seconds <= args.budget:
            return True
        skipped.append(f"{name} (needs ~{seconds:.0f} s, {elapsed():.0f} s of {args.budget:.0f} s used)")
        log(f"[bench] skipped {skipped[-1]}")
        return False

    nbytes = lgf.lgf_required_bytes(dims, home)
    pristine = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    work = torch.empty_like(pristine)
    hp = lgf.lgf_create(dims, home, stream, pristine)
    lgf.lgf_generate_links(hp, seed, eps, True)
    hw = lgf.lgf_create(dims, home, stream, work)
    work.copy_(pristine)
    # the fixed-link sweep variants picked on this lattice and GPU
    lgf.lgf_autotune_fixed(hw, finish, 4)
    lgf.lgf_autotune_fixed(hw, bulk, 4)
    torch.cuda.synchronize()
    fixed_tuning = {f: lgf.lgf_get_fixed_tuning(hw, f) for f in (bulk, finish)}
    log(f"[bench] {dims} V={V} generated; field {nbytes / 1e9:.2f} GB; fixed-link tuning {FIXED_TUNING_KEYS} "
        f"fp64-12 {fixed_tuning[finish]} fp32-12 {fixed_tuning[bulk]}; {elapsed():.1f} s")

    # ---- the timed steps: check intervals of the FP64 gauge fixing
    lgf.lgf_fix_begin(hw, finish)
    sweep0 = 0
    for w in range(args.warmup):
        F, th, ms = lgf.lgf_fix_chunk(hw, chunk, omega, 0.0, 0, sweep0)
        sweep0 += chunk
        log(f"[bench] warmup {w}: F {F:.12f} theta {th:.3e}, sweeps {ms:.1f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = []
    for _ in range(args.steps):
        steps.append(lgf.lgf_fix_chunk(hw, chunk, omega, 0.0, 0, sweep0))
        sweep0 += chunk
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lgf.lgf_fix_end(hw)
    step_s = t1 - t0
    sweep_ms = sum(r[2] for r in steps)
    launch_ms = sweep_ms / (2 * chunk * args.steps)
    log(f"[bench] {args.steps} steps in {step_s * 1e3:.1f} ms ({step_s / args.steps * 1e3:.2f} ms per step); "
        f"sweep kernels {launch_ms:.4f} ms per launch; theta {steps[-1][1]:.3e}")

    # the mixed form's bulk sweep (FP32-12 links and g, its autotuned variant)
    # in a session of its own, against the step's FP64 sweep
    lgf.lgf_fix_begin(hw, bulk)
    lgf.lgf_fix_chunk(hw, chunk, omega, 0.0, 0, 0)
    bulk_ms = sum(lgf.lgf_fix_chunk(hw, chunk, omega, 0.0, 0, chunk * (k + 1))[2] for k in range(5)) / (10 * chunk)
    lgf.lgf_fix_end(hw)
    mixed_bulk = mixed_bulk_summary(bulk, fixed_tuning[bulk], Vh, bulk_ms, launch_ms)
    log(f"[bench] mixed bulk sweep: {json.dumps(mixed_bulk)}")

    # roofline of the dominant kernel (the step's sweep), from the HIP events
    # the library records around each chunk's sweeps on the launch stream
    lanes, block, order, layout = fixed_tuning[finish]
    by = Vh * fixed_site_bytes(finish)
    achieved = by / (launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(fixed_traffic_key(finish, lanes, block, order, layout, dims))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": f"fixed_sweep_kernel<fp64-12, lanes/site {lanes}> block {block}, tile order "
                          f"{TILE_ORDERS[order]}, links from the {LINK_LAYOUTS[layout]}",
                "avg_launch_ms": round(launch_ms, 4), "launches": 2 * chunk * args.steps,
                "bytes_per_launch": by,
                "basis": f"{Vh} site updates per launch x {fixed_site_bytes(finish)} B: the fixed-link form "
                         f"reads the 8 links of a site, reads and writes g(x) and reads the neighbouring g of "
                         f"the other parity once (96 B each, FP64-12); the link-rewriting sweep moves 2304 B "
                         f"per update in FP64-18, 1536 B in FP64-12"}
    if traffic:
        roofline["traffic_GBs"] = round(traffic / (launch_ms * 1e-3) / 1e9, 1)
        roofline["traffic_frac"] = round(roofline["traffic_GBs"] / HBM_PEAK_GBS, 4)
        roofline["traffic_over_algorithmic"] = round(traffic / by, 4)
    copy_gbs = lgf.lgf_copy_bandwidth(4 << 30, 10, stream)
    roofline["copy_ceiling_GBs"] = round(copy_gbs, 1)
    roofline["frac_of_copy_ceiling"] = round(achieved / copy_gbs, 4)
    log(f"[bench] copy ceiling {copy_gbs:.1f} GB/s; step sweep kernel at {achieved:.1f} GB/s; {elapsed():.1f} s")

    # ---- time to theta < 1e-14, each form once on the same input
    extras = {}

    def fix_once(name, params, tuned=None):
        work.copy_(pristine)
        st, r, _ = lgf.lgf_gauge_fix(hw, params)
        e = {"status": lgf.STATUS_NAMES.get(int(st), int(st)), "time_to_theta_s": r["t_total_ms"] / 1e3,
             "sweeps": r["sweeps"], "sweeps_bulk": r["sweeps_bulk"], "theta": r["theta"], "F": r["F"],
             "site_updates_per_s": V * r["sweeps"] / (r["t_total_ms"] / 1e3),
             "t_sweep_bulk_s": r["t_sweep_bulk_ms"] / 1e3, "t_sweep_finish_s": r["t_sweep_finish_ms"] / 1e3,
             "t_measure_s": r["t_measure_ms"] / 1e3, "t_convert_s": r["t_convert_ms"] / 1e3}
        if tuned:
            e["tuning"] = tuned
        extras[name] = e
        log(f"[bench] {name}: {json.dumps(e)}; {elapsed():.1f} s")
        return e

    time_to_theta = {}
    cpu = None
    if not args.no_extras:
        pm = lgf.fix_params(omega=omega, theta_target=theta_target, theta_switch=theta_switch, bulk_format=bulk,
                            finish_format=finish, fixed_links=1)
        mixed = fix_once("mixed_fp32-12_bulk_fp64-12_finish", pm)
        time_to_theta["mixed_s"] = mixed["time_to_theta_s"]
        est = 1.3 * mixed["t_sweep_finish_s"] * mixed["sweeps"] / max(mixed["sweeps"] - mixed["sweeps_bulk"], 1)
        if fits("plain FP64 time-to-theta", est + args.cpu_seconds + 40.0):
            p64 = lgf.fix_params(omega=omega, theta_target=theta_target, bulk_format=finish, finish_format=finish,
                                 fixed_links=1)
            plain = fix_once("fp64_fp64-12", p64)
            time_to_theta["fp64_s"] = plain["time_to_theta_s"]
            time_to_theta["mixed_speedup_vs_fp64"] = plain["time_to_theta_s"] / mixed["time_to_theta_s"]
            time_to_theta["dF_mixed_vs_fp64"] = mixed["F"] - plain["F"]
        # the same mixed form leaving FP32 three decades later (its bulk reaches
        # about 9e-13 on this field before rounding stops it)
        if fits("mixed time-to-theta with the switch at 1e-11", 0.9 * mixed["time_to_theta_s"] + args.cpu_seconds + 40):
            pl = lgf.fix_params(omega=omega, theta_target=theta_target, theta_switch=LOW_SWITCH, bulk_format=bulk,
                                finish_format=finish, fixed_links=1)
            low = fix_once("mixed_fp32-12_bulk_to_1e-11_fp64-12_finish", pl)
            time_to_theta["mixed_switch_1e-11_s"] = low["time_to_theta_s"]
            if "fp64_s" in time_to_theta:
                time_to_theta["mixed_switch_1e-11_speedup_vs_fp64"] = time_to_theta["fp64_s"] / low["time_to_theta_s"]
                time_to_theta["dF_mixed_switch_1e-11_vs_fp64"] = low["F"] - plain["F"]
    # the CPU baseline before the optional runs (the line needs it)
    if not args.no_cpu_baseline and fits("cpu_baseline", args.cpu_seconds + 40.0):
        log("[bench] timing the FP64 oracle on the host")
        cpu = cpu_baseline(dims, seed, eps, omega, args.cpu_sweeps, args.cpu_seconds)
        log(f"[bench] cpu_baseline: {json.dumps(cpu)}; {elapsed():.1f} s")
    # the batched form: 48 lattices of 8^4..24^4 in one persistent launch per
    # parity, against one launch per lattice and against plain FP64
    batched = None
    if not args.no_extras and fits("the 48-configuration ensemble", 45.0):
        ens = ensemble_bench(lgf, stream)
        extras["ensemble48"] = ens
        batched = batched_summary(ens)
        log(f"[bench] ensemble: {json.dumps(batched)}; {elapsed():.1f} s")
    if not args.no_extras and "mixed_s" in time_to_theta:
        # the finish on the split copy of the links (FP64 arithmetic; links
        # within 2^-40, so a sweep is within ~1e-11 of the FP64 one, not 1e-12)
        if fits("mixed time-to-theta with the split finish", 1.1 * time_to_theta["mixed_s"]):
            lgf.lgf_autotune_fixed(hw, split, 4)
            ps = lgf.fix_params(omega=omega, theta_target=theta_target, theta_switch=theta_switch, bulk_format=bulk,
                                finish_format=split, fixed_links=1)
            rs = fix_once("mixed_fp32-12_bulk_fp64-12s_finish", ps)
            time_to_theta["mixed_split_finish_s"] = rs["time_to_theta_s"]
            time_to_theta["dF_mixed_split_vs_mixed"] = rs["F"] - mixed["F"]
        # the paper's form: FP64 18-real links rewritten by every update
        if fits("plain FP64-18 link-rewriting time-to-theta", 150.0):
            p18 = lgf.fix_params(omega=omega, theta_target=theta_target)
            r18 = fix_once("fp64_18_link_sweeps", p18,
                           tuned=dict(zip(lgf.TUNING_FIELDS, lgf.lgf_get_tuning(hw, home))))
            time_to_theta["fp64_18_link_sweeps_s"] = r18["time_to_theta_s"]
            time_to_theta["mixed_speedup_vs_fp64_18_link_sweeps"] = r18["time_to_theta_s"] / mixed["time_to_theta_s"]
    lgf.lgf_destroy(hw)
    lgf.lgf_destroy(hp)
    del work, pristine
    torch.cuda.empty_cache()
    if not args.no_extras and fits("overrelaxation kernels at 32^4", 30.0):
        extras["or_kernel_32x4"] = or_kernels_32x4(lgf, stream, 1.7)
        log(f"[bench] 32^4 overrelaxation kernels: {json.dumps(extras['or_kernel_32x4'])}; {elapsed():.1f} s")
    if not args.no_extras:
        # the small 8^4 workload to theta < 1e-12, plain FP64-18 (its oracle time is in cpu_baseline)
        h8 = lgf.lgf_create((8, 8, 8, 8), home, stream)
        lgf.lgf_generate_links(h8, 0, 0.25, True)
        p8 = lgf.fix_params(omega=1.7, theta_target=1e-12)
        lgf.lgf_synchronize(h8)
        st8, r8, _ = lgf.lgf_gauge_fix(h8, p8)
        lgf.lgf_destroy(h8)
        extras["gauge_8x4"] = {"status": int(st8), "sweeps": r8["sweeps"],
                               "time_to_theta_s": r8["t_total_ms"] / 1e3, "theta": r8["theta"]}

    out = {
        "metric": "OR site-updates/s at 64^4 (FP64 check intervals of the Landau gauge fixing); "
                  "time-to-theta<1e-14 mixed vs FP64",
        "value": V * chunk * args.steps / step_s,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, dims))} SU(3) Landau overrelaxation (omega {omega}): one step = "
                               f"{chunk} full sweeps of the fixed-link form (FP64 arithmetic, links and g in "
                               f"FP64 12-real storage, the links read from the {LINK_LAYOUTS[layout]}) from a "
                               f"hipGraph + FP64 reunitarization of g + FP64 F/theta measurement",
                   "dims": list(dims), "seed": seed, "eps": eps, "haar": True, "omega": omega,
                   "sweeps_per_step": chunk, "theta_after_steps": steps[-1][1],
                   "fixed_sweep_tuning": {lgf.FORMAT_NAMES[f]: dict(zip(FIXED_TUNING_KEYS, t))
                                          for f, t in fixed_tuning.items()}},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_theta": time_to_theta,
        "mixed_bulk": mixed_bulk,
        "batched": batched,
        "extras": extras,
        "skipped": skipped,
        "wall_s": round(elapsed(), 1),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
