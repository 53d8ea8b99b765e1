#!/usr/bin/env python3
"""Benchmark of the HashPoint hot path on one MI355X.

A step is one pass of the whole path over one view: pixel-table build,
search + primary-surface sampling, and decode + composite.  Workload: the
object-scale scene (1M points on 12 random spheres, boxes and tori in
[-1, 1]^3, 32-dim features), one 800x800 view at 40 deg from distance 4,
r = 0.01, K = 8, 16 samples per ray, decoder 32-64-64-4.  `value` is for the
BF16 decoder; the FP32 decoder is timed the same way (`value_fp32`).  RGB
errors are max abs against the oracle's binary64 render on a ray sample.

Prints one JSON line.  Inputs are resident in device memory before timing.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s (search+sample+render) at 800x800, 1M pts; BF16 vs FP32 at stated RGB error"
HBM_PEAK_GBS = 8000.0


def search_algorithmic_bytes(n_buckets, n_in, n_rays, s_tot, K):
    """Bytes the search + sampling stage must move at minimum: the table
    (offsets 8 B per bucket, one 16 B entry per inserted point), 16 B of
    per-ray outputs, and per selected sample its t and K (index, distance)."""
    return 8 * n_buckets + 16 * n_in + 16 * n_rays + (4 + 8 * K) * s_tot


def build_algorithmic_bytes(n, n_in, n_buckets):
    """Table build: read xyz (12 B per point), write one 16 B entry and a
    4 B index per inserted point plus a 4 B slot per point, and 8 B of
    offsets and depth summary per bucket."""
    return 12 * n + 24 * n_in + 8 * n_buckets


def render_algorithmic_bytes(s_tot, K, n_used, n_rays, C=32):
    """Render: every sample's t and K (index, distance), the features of every
    point a sample uses (read once), 20 B of outputs per ray."""
    return (4 + 8 * K) * s_tot + 4 * C * n_used + 20 * n_rays


MLP_FLOP_PER_SAMPLE = 2 * (32 * 64 + 64 * 64 + 64 * 4)   # 12,800
CHIP_CUS, CHIP_GHZ = 256, 2.4
MFMA_BF16_PEAK_TFLOPS = 2500.0
COUNTERS_FILE = os.path.join(ROOT, "profiles", "forward_path_objects_1m.md")
RENDER_KERNEL = "k_render_shared<1,16>"  # the default BF16 render launch (HP_BF16 = 1)
COUNTER_SOURCES = ("paper_2404_14044_amd/csrc", "include")


def sources_sha():
    """Hash of every source file the kernels are built from: counters taken
    on another build describe another kernel."""
    import hashlib
    h = hashlib.sha256()
    for d in COUNTER_SOURCES:
        base = os.path.join(ROOT, d)
        for name in sorted(os.listdir(base)):
            if name.endswith((".hip", ".hpp", ".h")):
                h.update(name.encode())
                with open(os.path.join(base, name), "rb") as f:
                    h.update(f.read())
    return h.hexdigest()[:16]


def load_counters():
    """Per-kernel counter figures from the committed profile summary, or None
    when they were taken on other sources than the ones built here."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    text = open(COUNTERS_FILE).read()
    i = text.find("```json")
    if i < 0:
        return None
    j = text.find("```", i + 7)
    data = json.loads(text[i + 7:j])
    return data if data.get("sources_sha") == sources_sha() else None


def pct(a, q):
    return float(np.percentile(np.asarray(a, np.float64), q))


def dist_stats(a):
    return {"mean": float(np.mean(a)), "median": pct(a, 50), "p10": pct(a, 10), "p90": pct(a, 90)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target wall time of the oracle CPU baseline (0 = skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--layout", type=int, default=0)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip every extra leg (batched views, training step, ...)")
    ap.add_argument("--legs", default="all",
                    help="comma-separated extra legs to run (batched, train, radius, samplers, "
                         "samplers_room, knp, fused, room, sweep) or 'all'")
    ap.add_argument("--summarize", nargs="+", metavar="DIR",
                    help="print the markdown summary of rocprofv3 output directories "
                         "(kernel stats and counter collections) and exit; no GPU used")
    args = ap.parse_args()

    if args.summarize:
        print(summarize_profiles(args.summarize))
        return

    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(views would shard across GPUs with no exchange in the forward pass)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2404_14044_amd import hashpoint as hp
    from paper_2404_14044_amd import scenes

    dev = torch.device("cuda:0")
    sc = scenes.objects_1m()
    cam = sc.cams[0]
    p = sc.params.replace(layout=args.layout)
    xyz = torch.from_numpy(sc.xyz).to(dev)
    feat = torch.from_numpy(sc.feat).to(dev)
    mlp = hp.to_device_mlp(sc.mlp, dev)
    R = cam.W * cam.H
    ws = torch.empty(hp.table_workspace(xyz.shape[0], [cam], p), dtype=torch.uint8, device=dev)
    smp = hp.alloc_samples(R, p, dev)
    outs = {prec: {"rgb": torch.empty(R * 3, device=dev), "depth": torch.empty(R, device=dev),
                   "acc": torch.empty(R, device=dev)} for prec in (hp.HP_FP32, hp.HP_BF16)}
    # the stream every launch below goes to; the events are recorded on it
    stream = torch.cuda.current_stream()

    def step(prec, ev=None):
        if ev: ev[0].record(stream)
        tab = hp.build_table(xyz, [cam], p, ws=ws, stream=stream)
        if ev: ev[1].record(stream)
        hp.search_sample(tab, p, out=smp, stream=stream)
        if ev: ev[2].record(stream)
        hp.render(smp, R, feat, mlp, p, prec, out=outs[prec], stream=stream)
        if ev: ev[3].record(stream)
        return tab

    def timed(prec):
        for _ in range(args.warmup):
            step(prec)
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
        t0 = time.perf_counter()
        for k in range(args.steps):
            tab = step(prec, evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3]),
                        e[0].elapsed_time(e[3])] for e in evs])
        return wall, st, tab

    wall16, st16, tab = timed(hp.HP_BF16)
    wall32, st32, _ = timed(hp.HP_FP32)

    offs = tab.offsets()
    n_in = int(offs[-1].item())
    n_sel = smp["n_sel"].cpu().numpy()
    s_tot = int(n_sel.sum())
    hit_rays = int((smp["n_nbr"] > 0).sum().item())
    ki = smp["knn_idx"].view(R, p.n_samples, p.K)
    mask = torch.arange(p.n_samples, device=dev)[None, :] < smp["n_sel"][:, None]
    used = torch.unique(ki[mask].reshape(-1))
    n_used = int((used >= 0).sum().item())

    ms16 = wall16 * 1e3 / args.steps
    ms32 = wall32 * 1e3 / args.steps
    build_ms = float(np.mean(st16[:, 0]))
    search_ms = float(np.mean(st16[:, 1]))
    render_ms = float(np.mean(st16[:, 2]))
    a_bytes = search_algorithmic_bytes(tab.n_buckets, n_in, R, s_tot, p.K)
    achieved = a_bytes / (search_ms * 1e-3) / 1e9
    b_bytes = build_algorithmic_bytes(int(xyz.shape[0]), n_in, tab.n_buckets)
    r_bytes = render_algorithmic_bytes(s_tot, p.K, n_used, R)
    mlp_tflops = MLP_FLOP_PER_SAMPLE * s_tot / (render_ms * 1e-3) / 1e12

    result = {
        "metric": METRIC,
        "value": R / (ms16 * 1e-3) / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms16,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "objects_1m: 1M surface points (12 random spheres/boxes/tori, "
                               "seed 2), one 800x800 view, hfov 40, r=0.01, K=8, S=16, "
                               "t in [2, 6], decoder 32-64-64-4 BF16 on MFMA",
                   "rays": R, "points": int(xyz.shape[0]), "layout": args.layout},
        "value_fp32": R / (ms32 * 1e-3) / 1e6,
        "ms_per_step_fp32": ms32,
        "step_ms_bf16": dist_stats(st16[:, 3]),
        "step_ms_fp32": dist_stats(st32[:, 3]),
        "stage_ms_bf16": {"build": dist_stats(st16[:, 0]), "search_sample": dist_stats(st16[:, 1]),
                          "render": dist_stats(st16[:, 2])},
        "stage_ms_fp32": {"build": dist_stats(st32[:, 0]), "search_sample": dist_stats(st32[:, 1]),
                          "render": dist_stats(st32[:, 2])},
        "workload_stats": {"n_in": n_in, "n_buckets": int(tab.n_buckets), "samples": s_tot,
                           "rays_with_neighbours": hit_rays,
                           "rays_with_samples": int((n_sel > 0).sum()), "points_used": n_used},
        "roofline": {"kernel": "k_search_sample", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "algorithmic_bytes": a_bytes},
        "rooflines_other": {
            "build": {"kernels": "k_build_begin .. k_sort_listed (one build, two-level)", "bound": "hbm",
                      "algorithmic_bytes": b_bytes, "achieved": b_bytes / (build_ms * 1e-3) / 1e9,
                      "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": b_bytes / (build_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "render_bf16": {"kernel": RENDER_KERNEL, "bound": "hbm",
                            "algorithmic_bytes": r_bytes,
                            "achieved": r_bytes / (render_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": r_bytes / (render_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                            "decoder_tflops": mlp_tflops,
                            "decoder_frac_of_bf16_mfma_peak": mlp_tflops / MFMA_BF16_PEAK_TFLOPS},
        },
    }
    counters = load_counters()
    if counters is not None:
        ks = counters["kernels"].get("k_search_sample_k8")
        if ks:
            traffic = (ks["FETCH_SIZE_kib"] * counters["fetch_scale"]
                       + ks["WRITE_SIZE_kib"] * counters["write_scale"]) * 1024.0
            result["roofline"]["traffic"] = traffic
            result["roofline"]["traffic_over_algorithmic"] = traffic / a_bytes
            slots = search_ms * 1e-3 * CHIP_GHZ * 1e9 * CHIP_CUS
            result["roofline"]["measured_limiter"] = {
                "resource": "VALU issue (one wave64 VALU instruction per CU per cycle)",
                "valu_insts": ks["SQ_INSTS_VALU"], "salu_insts": ks.get("SQ_INSTS_SALU"),
                "valu_issue_frac": ks["SQ_INSTS_VALU"] / slots,
                "valu_insts_per_ray_with_neighbours": ks["SQ_INSTS_VALU"] / max(hit_rays, 1)}
        kr = counters["kernels"].get(RENDER_KERNEL)
        if kr and "SQ_INSTS_MFMA" in kr:
            rr = result["rooflines_other"]["render_bf16"]
            rr["mfma_insts"] = kr["SQ_INSTS_MFMA"]
            # a 16x16x32 BF16 product is 16 cycles of one SIMD's matrix core
            simd_cycles = render_ms * 1e-3 * CHIP_GHZ * 1e9 * CHIP_CUS * 4
            rr["mfma_busy_frac"] = kr["SQ_INSTS_MFMA"] * 16 / simd_cycles
            rr["valu_issue_frac"] = kr["SQ_INSTS_VALU"] / (simd_cycles / 4)
            rr["vmem_read_insts"] = kr.get("SQ_INSTS_VMEM_RD")
        result["roofline"]["counters_from"] = os.path.relpath(COUNTERS_FILE, ROOT)
    # achievable bandwidth on this machine: a plain 1 GiB device-to-device copy
    copy_gbs = copy_bandwidth_gbs(dev)
    result["roofline"]["copy_gbs"] = copy_gbs
    result["roofline"]["frac_of_copy"] = achieved / copy_gbs

    if args.calibrate_copy:
        src = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    if not args.no_extra:
        legs = [("batched", "batched_16", lambda: batched_leg(sc)),
                ("train", "train_4x400", lambda: train_leg(sc)),
                ("radius", "radius_modes", lambda: radius_modes_leg(sc)),
                ("samplers", "samplers", lambda: sampler_leg(sc, ms_steps=400)),
                ("samplers_room", "samplers_room_5m", room_sampler_leg),
                ("knp", "knp", lambda: knp_leg(sc)),
                ("fused", "fused", lambda: fused_leg(sc)),
                ("room", "room_5m", room_leg),
                ("sweep", "complexity_sweep", scaling_leg)]
        wanted = set(l for l, _, _ in legs) if args.legs == "all" else set(args.legs.split(","))
        unknown = wanted - set(l for l, _, _ in legs)
        if unknown:
            print(f"bench.py: unknown legs {sorted(unknown)}", file=sys.stderr)
            sys.exit(2)
        for name, key, fn in legs:
            if name in wanted:
                print(f"bench.py: leg {name}", file=sys.stderr, flush=True)
                result[key] = fn()

    if args.cpu_seconds > 0:
        result.update(cpu_leg(sc, p, smp, outs, R, args.cpu_seconds))

    print(json.dumps(result), flush=True)


def kernel_key(name):
    """Short name of a kernel as the profiler reports it: no return type,
    namespace or argument list; template arguments kept, without spaces
    (e.g. "k_render_bf16<32,false>")."""
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    depth, cut = 0, len(name)
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    name = name[:cut]
    head, sep, tmpl = name.partition("<")
    head = head.split("::")[-1]
    return (head + sep + tmpl).replace(" ", "")


def summarize_profiles(dirs):
    """Markdown summary of rocprofv3 runs: kernel statistics (calls, average
    duration) from *_kernel_stats.csv and, from *_counter_collection.csv,
    every counter's mean value per dispatch, by kernel.  The json block at the
    end is what the bench line reads (with the hash of the sources)."""
    import csv
    stats, ctr = {}, {}
    for d in dirs:
        for root, _, files in os.walk(d):
            for f in files:
                path = os.path.join(root, f)
                if f.endswith("kernel_stats.csv"):
                    with open(path) as fh:
                        for row in csv.DictReader(fh):
                            stats[kernel_key(row["Name"])] = {"calls": int(row["Calls"]),
                                                  "avg_us": float(row["AverageNs"]) / 1e3,
                                                  "total_us": float(row["TotalDurationNs"]) / 1e3}
                elif f.endswith("counter_collection.csv"):
                    with open(path) as fh:
                        for row in csv.DictReader(fh):
                            k = kernel_key(row["Kernel_Name"])
                            ent = ctr.setdefault(k, {}).setdefault(row["Counter_Name"], {})
                            did = (path, row["Dispatch_Id"])
                            ent[did] = ent.get(did, 0.0) + float(row["Counter_Value"])
    out = ["| kernel | calls | avg µs | total µs |", "|---|---|---|---|"]
    for name, v in sorted(stats.items(), key=lambda kv: -kv[1]["total_us"]):
        out.append(f"| `{name[:60]}` | {v['calls']} | {v['avg_us']:.1f} | "
                   f"{v['total_us']:.1f} |")
    names = sorted({c for k in ctr.values() for c in k})
    out += ["", "| kernel | " + " | ".join(names) + " |", "|---" * (len(names) + 1) + "|"]
    per_kernel = {}
    for k in sorted(ctr):
        vals = {}
        for c in names:
            d = ctr[k].get(c)
            if d:
                vals[c] = sum(d.values()) / len(d)
        per_kernel[k] = {(c + "_kib" if c in ("FETCH_SIZE", "WRITE_SIZE") else c): v
                         for c, v in vals.items()}
        out.append(f"| `{k[:60]}` | " + " | ".join(f"{vals[c]:.4g}" if c in vals else "-"
                                                   for c in names) + " |")
    # calibration: the largest device copy in the runs is the 1 GiB copy that
    # measures the box's bandwidth (1 GiB read, 1 GiB written)
    scale = {"FETCH_SIZE": None, "WRITE_SIZE": None}
    for k in ctr:
        if "copyBuffer" not in k:
            continue
        for c in scale:
            if c in ctr[k]:
                scale[c] = float(1 << 30) / (max(ctr[k][c].values()) * 1024.0)
    out += ["", f"Calibration (largest device copy, 1 GiB each way): FETCH_SIZE x "
                f"{scale['FETCH_SIZE']}, WRITE_SIZE x {scale['WRITE_SIZE']}.",
            "", "```json", json.dumps({"sources_sha": sources_sha(),
                                        "fetch_scale": scale["FETCH_SIZE"],
                                        "write_scale": scale["WRITE_SIZE"],
                                        "kernels": per_kernel}, indent=1),
            "```"]
    return "\n".join(out)


def copy_bandwidth_gbs(dev, nbytes=1 << 30, reps=5):
    """Read + write bytes per second of a device-to-device copy (the box's
    achievable HBM bandwidth), best of `reps`."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def _time_ms(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def batched_leg(sc, reps=5):
    """16 views of the object scene, sides uniform in {256..1024}: one batched
    pass (eager and replayed from a captured graph) vs 16 per-view passes,
    with the library's default layout and launch shapes and with the
    autotuner's choice for these views (tuned here, in a fresh cache)."""
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    from paper_2404_14044_amd import scenes
    from paper_2404_14044_amd.autotune import Autotuner
    from paper_2404_14044_amd.batched import BatchedRenderer, render_views_separately
    dev = torch.device("cuda:0")
    bs = scenes.batched_16(base=sc)
    xyz = torch.from_numpy(bs.xyz).to(dev)
    feat = torch.from_numpy(bs.feat).to(dev)
    mlp = hp.to_device_mlp(bs.mlp, dev)
    rays = sum(c.W * c.H for c in bs.cams)
    out = {"rays": rays, "views": len(bs.cams)}
    tuner = Autotuner()
    t0 = time.time()
    tuned = BatchedRenderer(xyz, feat, mlp, bs.cams, bs.params, hp.HP_BF16, tuner=tuner)
    ent = tuner.entry(xyz, bs.cams, bs.params, hp.HP_BF16)
    out["autotune"] = {"best": ent["best"], "trials": len(ent["trials"]),
                       "tune_s": time.time() - t0,
                       "frame_ms_default": ent["default_ms"], "frame_ms_tuned": ent["ms"]}
    for name, br in (("default", BatchedRenderer(xyz, feat, mlp, bs.cams, bs.params, hp.HP_BF16)),
                     ("tuned", tuned)):
        t_eager = _time_ms(br.run_eager, reps)
        br.capture()
        t_graph = _time_ms(br.replay, reps)
        state = render_views_separately(xyz, feat, mlp, bs.cams, br.params, hp.HP_BF16)
        t_sep = _time_ms(lambda: render_views_separately(xyz, feat, mlp, bs.cams, br.params,
                                                         hp.HP_BF16, state), reps)
        out[name] = {"graph_ms": t_graph, "eager_ms": t_eager, "separate_ms": t_sep,
                     "graph_mrays_s": rays / t_graph / 1e3, "eager_mrays_s": rays / t_eager / 1e3,
                     "separate_mrays_s": rays / t_sep / 1e3,
                     "speedup_vs_separate": t_sep / t_graph}
        del br, state
    out["tuned_over_default_graph"] = out["default"]["graph_ms"] / out["tuned"]["graph_ms"]
    return out


def radius_modes_leg(sc, reps=5):
    """Build + search/sample + render (BF16) on the same view under each search
    radius law: the fixed radius, the linear cone equal to r at t_near, and the
    per-pixel cone of Eq. 3 with its two small-angle variants (rddot puts the
    principal pixel's radius at t_near equal to r).  Reports the guard band g
    the search uses next to the paper's kernel size s."""
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    from paper_2404_14044_amd import scenes
    dev = torch.device("cuda:0")
    cam = sc.cams[0]
    R = cam.W * cam.H
    xyz = torch.from_numpy(sc.xyz).to(dev)
    feat = torch.from_numpy(sc.feat).to(dev)
    mlp = hp.to_device_mlp(sc.mlp, dev)
    base = sc.params
    modes = {
        "fixed": base,
        "linear_cone": base.replace(inv_tref=float(np.float32(1.0 / base.t_near))),
    }
    for name, m in (("eq3", hp.HP_RADIUS_EQ3), ("eq3_af", hp.HP_RADIUS_EQ3_AF),
                    ("eq3_ae", hp.HP_RADIUS_EQ3_AE)):
        modes[name] = base.replace(radius_mode=m, rddot=scenes.eq3_rddot(m, base.radius, base.t_near))
    out = {}
    for name, p in modes.items():
        ws = torch.empty(hp.table_workspace(xyz.shape[0], [cam], p), dtype=torch.uint8, device=dev)
        smp = hp.alloc_samples(R, p, dev)
        o = {"rgb": torch.empty(R * 3, device=dev)}
        holder = {}

        def build():
            holder["tab"] = hp.build_table(xyz, [cam], p, ws=ws)

        t_build = _time_ms(build, reps)
        tab = holder["tab"]
        t_search = _time_ms(lambda: hp.search_sample(tab, p, out=smp), reps)
        t_render = _time_ms(lambda: hp.render(smp, R, feat, mlp, p, hp.HP_BF16, out=o), reps)
        n_nbr = smp["n_nbr"].float()
        g, _ = hp.view_bounds(cam, p)
        total = t_build + t_search + t_render
        out[name] = {"build_ms": t_build, "search_ms": t_search, "render_ms": t_render,
                     "mrays_s": R / total / 1e3, "guard_g": g,
                     "paper_s": hp.paper_kernel_size(cam, p),
                     "mean_n_nbr": float(n_nbr.mean().item()),
                     "overflow_frac": float((smp["flags"] & 1).float().mean().item()),
                     "samples": int(smp["n_sel"].sum().item())}
        del ws, smp, o, tab, holder
    return out


def sampler_leg(sc, ms_steps, reps=5):
    """Primary-surface walk at several gamma (Sec. 3.3 and the supplement's
    gamma sweep: smaller gamma samples further past the primary surface) and
    the uniform multi-surface baseline (Sec. 3.5; ms_steps positions over
    [t_near, t_far], about one per search radius, each with its own radius
    search over all of the ray's neighbours), all with up to 64 samples per
    ray except the workload's own gamma = 0.9, S = 16.  Build + search/sample
    + render (BF16) on the same view."""
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    dev = torch.device("cuda:0")
    cam = sc.cams[0]
    R = cam.W * cam.H
    xyz = torch.from_numpy(sc.xyz).to(dev)
    feat = torch.from_numpy(sc.feat).to(dev)
    mlp = hp.to_device_mlp(sc.mlp, dev)
    base = sc.params
    runs = {f"ps_gamma0.9_S{base.n_samples}": base}
    for gm in (0.9, 0.5, 0.1, 0.01):
        runs[f"ps_gamma{gm}_S64"] = base.replace(gamma=float(np.float32(gm)), n_samples=64)
    ms_name = f"ms_{ms_steps}_S64"
    runs[ms_name] = base.replace(sampler=hp.HP_SAMPLER_MS, ms_steps=ms_steps, n_samples=64)
    out = {"rays": R, "points": int(xyz.shape[0])}
    ws = torch.empty(hp.table_workspace(xyz.shape[0], [cam], base), dtype=torch.uint8, device=dev)
    tab = hp.build_table(xyz, [cam], base, ws=ws)
    t_build = _time_ms(lambda: hp.build_table(xyz, [cam], base, ws=ws), reps)
    for name, p in runs.items():
        smp = hp.alloc_samples(R, p, dev)
        o = {"rgb": torch.empty(R * 3, device=dev)}
        t_search = _time_ms(lambda: hp.search_sample(tab, p, out=smp), reps)
        t_render = _time_ms(lambda: hp.render(smp, R, feat, mlp, p, hp.HP_BF16, out=o), reps)
        ns = smp["n_sel"]
        hit = int((ns > 0).sum().item())
        tot = t_build + t_search + t_render
        out[name] = {"search_ms": t_search, "render_ms": t_render, "total_ms": tot,
                     "mrays_s": R / tot / 1e3, "samples": int(ns.sum().item()),
                     "samples_per_hit_ray": float(ns.sum().item()) / max(hit, 1),
                     "hit_rays": hit}
        del smp, o
    ms = out[ms_name]["total_ms"]
    for name in runs:
        out[name]["speedup_vs_ms"] = ms / out[name]["total_ms"]
    return out


def room_sampler_leg(reps=3):
    """The sampler comparison on the scene-scale room (1008 x 756, 5M points,
    rays crossing 2-8 surfaces; MS positions every 0.02 = r over [0.5, 21])."""
    from paper_2404_14044_amd import scenes
    return sampler_leg(scenes.room_5m(), ms_steps=1025, reps=reps)


def knp_leg(sc, reps=5):
    """K-NP extraction + Eq. 1 blending (the image-based consumers of the same
    table and search, NPLF-style K = 8 and Pointersect-style K = 40): build +
    search + blend per step, no decoder."""
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    from paper_2404_14044_amd import scenes
    dev = torch.device("cuda:0")
    cam = sc.cams[0]
    R = cam.W * cam.H
    xyz = torch.from_numpy(sc.xyz).to(dev)
    colors = torch.from_numpy(scenes.point_colors(sc.xyz.shape[0], 9)).to(dev)
    p = sc.params
    ws = torch.empty(hp.table_workspace(xyz.shape[0], [cam], p), dtype=torch.uint8, device=dev)
    tab = hp.build_table(xyz, [cam], p, ws=ws)
    t_build = _time_ms(lambda: hp.build_table(xyz, [cam], p, ws=ws), reps)
    out = {}
    for K in (8, 40):
        o = {"rgb": torch.empty(R * 3, device=dev), "cnt": torch.empty(R, dtype=torch.int32, device=dev)}
        t = _time_ms(lambda: hp.knp_blend(tab, p, K, colors, out=o), reps)
        out[f"K{K}"] = {"knp_ms": t, "total_ms": t_build + t, "mrays_s": R / (t_build + t) / 1e3,
                        "full_rays": int((o["cnt"] == K).sum().item())}
    return out


def scaling_leg(reps=3):
    """Complexity check of Sec. 3.5 (build O(n), lookup O(m q)): the object
    scene at n = 0.25M .. 4M points with one 800x800 view, then n = 1M with
    views of 200^2 .. 1600^2 rays.  Reports build and search/sample times
    and their per-point / per-ray costs."""
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    from paper_2404_14044_amd import scenes
    dev = torch.device("cuda:0")

    def run(n, res):
        sc = scenes.objects_1m(n=n, res=res)
        cam, p = sc.cams[0], sc.params
        xyz = torch.from_numpy(sc.xyz).to(dev)
        ws = torch.empty(hp.table_workspace(n, [cam], p), dtype=torch.uint8, device=dev)
        tab = hp.build_table(xyz, [cam], p, ws=ws)
        smp = hp.alloc_samples(tab.n_rays, p, dev)
        tb = _time_ms(lambda: hp.build_table(xyz, [cam], p, ws=ws), reps)
        tsr = _time_ms(lambda: hp.search_sample(tab, p, out=smp), reps)
        nn = smp["n_nbr"].float()
        res_d = {"n": n, "rays": tab.n_rays, "build_ms": tb, "search_ms": tsr,
                 "build_ns_per_point": tb * 1e6 / n, "search_ns_per_ray": tsr * 1e6 / tab.n_rays,
                 "mean_neighbours_per_ray": float(nn.mean().item())}
        del ws, tab, smp, xyz
        return res_d

    by_n = [run(n, 800) for n in (250_000, 500_000, 1_000_000, 2_000_000, 4_000_000)]
    by_m = [run(1_000_000, r) for r in (200, 400, 800, 1600)]
    return {"by_points": by_n, "by_rays": by_m}


def fused_leg(sc, reps=10):
    """Search + sampling + render in one launch (samples stay on chip) vs the
    two launches of the main step, BF16, same table."""
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    dev = torch.device("cuda:0")
    cam, p = sc.cams[0], sc.params
    R = cam.W * cam.H
    xyz = torch.from_numpy(sc.xyz).to(dev)
    feat = torch.from_numpy(sc.feat).to(dev)
    mlp = hp.to_device_mlp(sc.mlp, dev)
    tab = hp.build_table(xyz, [cam], p)
    smp = hp.alloc_samples(R, p, dev)
    o = {"rgb": torch.empty(R * 3, device=dev), "depth": torch.empty(R, device=dev),
         "acc": torch.empty(R, device=dev)}
    fo = {"rgb": torch.empty(R * 3, device=dev), "depth": torch.empty(R, device=dev),
          "acc": torch.empty(R, device=dev), "n_sel": None}

    def sep():
        hp.search_sample(tab, p, out=smp)
        hp.render(smp, R, feat, mlp, p, hp.HP_BF16, out=o)

    t_sep = _time_ms(sep, reps)
    t_fus = _time_ms(lambda: hp.search_render(tab, p, feat, mlp, hp.HP_BF16, out=fo), reps)
    same = bool(torch.equal(o["rgb"], fo["rgb"]))
    return {"separate_ms": t_sep, "fused_ms": t_fus, "fused_over_separate": t_fus / t_sep,
            "identical_rgb": same}


def room_leg(reps=5):
    """Scene-scale workload (5M points, 1008x756, K = 16, S = 16): build +
    search/sample + render (BF16)."""
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    from paper_2404_14044_amd import scenes
    dev = torch.device("cuda:0")
    sc = scenes.room_5m()
    cam, p = sc.cams[0], sc.params
    R = cam.W * cam.H
    xyz = torch.from_numpy(sc.xyz).to(dev)
    feat = torch.from_numpy(sc.feat).to(dev)
    mlp = hp.to_device_mlp(sc.mlp, dev)
    ws = torch.empty(hp.table_workspace(xyz.shape[0], [cam], p), dtype=torch.uint8, device=dev)
    smp = hp.alloc_samples(R, p, dev)
    o = {"rgb": torch.empty(R * 3, device=dev)}
    holder = {}

    def build():
        holder["tab"] = hp.build_table(xyz, [cam], p, ws=ws)

    tb = _time_ms(build, reps)
    tab = holder["tab"]
    ts = _time_ms(lambda: hp.search_sample(tab, p, out=smp), reps)
    tr = _time_ms(lambda: hp.render(smp, R, feat, mlp, p, hp.HP_BF16, out=o), reps)
    return {"rays": R, "points": int(xyz.shape[0]), "build_ms": tb, "search_ms": ts, "render_ms": tr,
            "mrays_s": R / (tb + ts + tr) / 1e3, "samples": int(smp["n_sel"].sum().item()),
            "overflow_frac": float((smp["flags"] & 1).float().mean().item()),
            "guard_g": hp.view_bounds(cam, p)[0]}


def train_leg(sc, reps=5):
    """Training step on 4 views of 400x400: BF16 forward, FP32 gradients for
    the 1M x 32 features and the decoder, L2 loss to a random target; the
    backward recomputes search and sampling."""
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    from paper_2404_14044_amd import scenes
    dev = torch.device("cuda:0")
    ds = scenes.diff_4x400(base=sc)
    xyz = torch.from_numpy(ds.xyz).to(dev)
    feat = torch.from_numpy(ds.feat).to(dev).requires_grad_(True)
    mlp = {k: v.requires_grad_(True) for k, v in hp.to_device_mlp(ds.mlp, dev).items()}
    target = torch.from_numpy(ds.extra["target"]).to(dev)
    tab = hp.build_table(xyz, ds.cams, ds.params)
    keys = ("W1", "b1", "W2", "b2", "W3", "b3")

    def step():
        feat.grad = None
        for k in keys:
            mlp[k].grad = None
        rgb = hp.HashPointRender.apply(feat, *[mlp[k] for k in keys], tab, ds.params, hp.HP_BF16)
        loss = ((rgb - target) ** 2).mean()
        loss.backward()

    t_step = _time_ms(step, reps)
    smp = hp.search_sample(tab, ds.params)
    t_fwd = _time_ms(lambda: hp.render(hp.search_sample(tab, ds.params, out=smp), tab.n_rays,
                                       feat.detach(), {k: v.detach() for k, v in mlp.items()},
                                       ds.params, hp.HP_BF16), reps)
    return {"rays": tab.n_rays, "step_ms": t_step, "forward_ms": t_fwd,
            "backward_ms": t_step - t_fwd, "step_mrays_s": tab.n_rays / t_step / 1e3}


def exact_outputs_match(smp, ex, pix, p):
    """Every exact output of the GPU search + sampling on rays `pix` equals the
    oracle's bit for bit: neighbour counts, overflow flags, sample counts,
    primary surface, sample t, nearest-neighbour indices and distances."""
    S, K = p.n_samples, p.K
    h = {k: smp[k].cpu().numpy() for k in ("n_nbr", "flags", "n_sel", "primary", "t",
                                            "knn_idx", "knn_dist")}
    res = {"n_nbr": np.array_equal(h["n_nbr"][pix], ex["n_nbr"]),
           "flags": np.array_equal(h["flags"][pix].astype(np.uint32), ex["flags"]),
           "n_sel": np.array_equal(h["n_sel"][pix], ex["n_sel"]),
           "primary": np.array_equal(h["primary"][pix], ex["primary"])}
    ns = ex["n_sel"]
    mask = np.arange(S)[None, :] < ns[:, None]
    t = h["t"].reshape(-1, S)[pix]
    ki = h["knn_idx"].reshape(-1, S, K)[pix]
    kd = h["knn_dist"].reshape(-1, S, K)[pix]
    res["t_bits"] = np.array_equal(t[mask].view(np.int32), ex["t"][mask].view(np.int32))
    res["knn_idx"] = np.array_equal(ki[mask], ex["knn_idx"][mask])
    res["knn_dist_bits"] = np.array_equal(kd[mask].view(np.int32), ex["knn_dist"][mask].view(np.int32))
    res["all"] = all(bool(v) for v in res.values())
    return {k: bool(v) for k, v in res.items()}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(sc, p, smp, outs, R, seconds):
    """Oracle (brute-force search, candidate walk, binary64 render) on a
    bounded random sample of the same rays, with every host thread and with
    one; also the GPU's exact outputs and RGB errors on that sample."""
    import oracle
    from paper_2404_14044_amd import hashpoint as hp
    cam = sc.cams[0]
    pc = oracle.to_camera(sc.xyz, cam)
    rng = np.random.default_rng(99)
    threads = oracle.num_threads()

    def run(pix):
        t0 = time.perf_counter()
        ex = oracle.exact(pc, cam, p, pix)
        ref = oracle.render64(pc, sc.feat, sc.mlp, cam, p, ex)
        return ex, ref, time.perf_counter() - t0

    probe = np.sort(rng.choice(R, 256, replace=False)).astype(np.int32)
    _, _, dt = run(probe)
    n = int(min(R, max(256, 256 * seconds / max(dt, 1e-3))))
    pix = np.sort(rng.choice(R, n, replace=False)).astype(np.int32)
    ex, ref, dt = run(pix)
    # one thread, on a sample sized for about a fifth of the time
    oracle.set_num_threads(1)
    try:
        n1 = int(max(64, n / max(threads, 1) / 5))
        pix1 = np.sort(rng.choice(R, n1, replace=False)).astype(np.int32)
        _, _, dt1 = run(pix1)
    finally:
        oracle.set_num_threads(threads)
    errs = {}
    for prec, name in ((hp.HP_BF16, "bf16"), (hp.HP_FP32, "fp32")):
        o = outs[prec]
        rgb = o["rgb"].cpu().numpy().reshape(-1, 3)[pix].astype(np.float64)
        dep = o["depth"].cpu().numpy()[pix].astype(np.float64)
        acc = o["acc"].cpu().numpy()[pix].astype(np.float64)
        errs[f"rgb_err_{name}"] = float(np.abs(rgb - ref["rgb"]).max())
        errs[f"depth_err_{name}"] = float(np.abs(dep - ref["depth"]).max())
        errs[f"acc_err_{name}"] = float(np.abs(acc - ref["acc"]).max())
        errs[f"rgb_err_p999_{name}"] = float(np.percentile(np.abs(rgb - ref["rgb"]), 99.9))
    errs["oracle_exact_match"] = exact_outputs_match(smp, ex, pix, p)
    model = cpu_model()
    return {"cpu_baseline": {"value": n / dt / 1e6, "unit": "Mrays/s", "cores": threads,
                             "kind": "oracle", "cpu_model": model,
                             "sample": f"{n} random rays of the 800x800 view (brute-force search "
                                       f"over all 1M points, candidate walk, binary64 render), "
                                       f"{dt:.1f} s on {threads} threads",
                             "one_thread": {"value": n1 / dt1 / 1e6, "unit": "Mrays/s",
                                            "sample": f"{n1} random rays, {dt1:.1f} s"}},
            **errs}


if __name__ == "__main__":
    main()
