#!/usr/bin/env python3
"""Benchmark: path samples/s of the wavefront and the megakernel on the
procedural ~1M-triangle scene at 1920x1080, 1 spp per frame, max depth 8,
Russian roulette from vertex 3, next-event estimation on; plus the adjoint
(path-replay backward) samples/s on the same scene at 512x512, 8 spp,
depth 6, roulette off.

One step = one frame of the wavefront pipeline (raygen, extend, shade,
shadow, accumulate over all bounces).  Inputs are resident in device memory
before timing starts.  Prints one JSON line.

Besides the headline (the wavefront with the hybrid tail, eight frames in
flight) the line carries: the pure wavefront (every bounce a separate
extend / shade / shadow launch over compacted queues) and the megakernel,
frame by frame and in flight; compaction against no compaction at depth 8
and 16; the roofline of every traversal kernel, of the megakernel and of
both adjoint kernels; short runs of the divergence workload (10M triangles,
64 material ids) and of the batched workload (64 jobs); and the oracle
timed on the host cores.
"""
import argparse
import json
import os
import platform
import sys
import time

# At least ten hardware queues for this process (HIP's default is four),
# read when HIP first initialises: the library then keeps eight frames in
# flight, one stream each, beside the caller's stream, and a batch four
# pools, without sharing queues.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or "4") < 10:
    os.environ["GPU_MAX_HW_QUEUES"] = "10"

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# fp32 vector peak: 256 CUs x 2.4 GHz x 64 lanes x 2 flops (one wave64 fused
# multiply-add per CU and cycle) = 78.6 TFLOP/s; packed FP32 (or dual issue)
# doubles it to 157.3, but this build disables packed FP32, so 78.6 is the
# reachable ceiling
FP32_PEAK_TFLOPS = 78.6
FP32_PEAK_PACKED_TFLOPS = 157.3
# algorithmic flops of traversal: a BVH4 node visit tests four child boxes
# (20 flops each: six plane distances of one fused multiply-add, three
# maxima, three minima, the slack multiply and the compare), a watertight
# ray/triangle test 40 (9 subtractions, 12 for the shear, 9 for the edge
# functions, 2 for the determinant, 8 for the scaled depth and the division)
FLOPS_PER_NODE = 80
FLOPS_PER_TRI = 40
# the launch parameters the autotuner chose on MI355X for the wavefront with
# three frames in flight and for the megakernel (kept so that profiles stay
# comparable across changes); the stage profile, the
# rooflines and the committed rocprofv3 profiles use them (bench.py --fixed)
FIXED_PARAMS = {"wave": {"block": 256, "grid_mult": 4, "stack_lds": 8, "tail_threshold": 1 << 18, "tail_bounce": 3},
                "mega": {"block": 256, "grid_mult": 4, "stack_lds": 8, "mega_waves": 5}}
# launch parameters of the backward (512x512, 8 spp, depth 6; measured on
# MI355X): the radiance replay as one kernel, or as the wavefront stages with
# the hybrid tail from bounce 4
ADJOINT_PARAMS = {"mega": {"block": 256, "grid_mult": 8, "stack_lds": 8},
                  "wave": {"block": 256, "grid_mult": 8, "stack_lds": 8, "tail_threshold": 1 << 18, "tail_bounce": 4},
                  # with kept intersections the first replay's extend and
                  # shadow stages, which run side by side, do best on half
                  # the lanes each (5.98 against 6.09 ms at grid_mult 8)
                  "wave_keep": {"block": 256, "grid_mult": 4, "stack_lds": 8, "tail_threshold": 1 << 18,
                                "tail_bounce": 4}}
# the pure wavefront: no hybrid tail, every bounce in separate stage launches
PURE = {"tail_threshold": 0, "tail_bounce": 0, "tail_spread": False}
# launch parameters of the divergence workload (4 spp, depth 16)
DIVERGENCE_PARAMS = {"wave": {"block": 256, "grid_mult": 8, "stack_lds": 8, "tail_threshold": 1 << 18, "tail_bounce": 6},
                     "mega": {"block": 256, "grid_mult": 4, "stack_lds": 8}}
# batch options for the 64-job workload (measured on MI355X; four pools need
# more than the default four hardware queues, set above)
BATCH_OPTS = {"pool_capacity": 1 << 23, "block": 256, "grid_mult": 8, "stack_lds": 8, "pools": 4}
W, H, SPP, DEPTH, RR = 1920, 1080, 1, 8, 3
PROFILE = "procedural1M_1080p"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """CPU model and core counts of this host (the oracle's baseline runs here)."""
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "nproc": aff, "cpu_count": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(scene, cam, budget_s=12.0, single_s=3.0):
    """The oracle (plain C, all host threads this process may use, at most
    16: the host share of one GPU on the MI355X boxes, whose harness sets
    OMP_NUM_THREADS=16) on whole frames 0, 1, 2, ... of the benchmark
    workload, split in 262144-pixel chunks, until the time budget is spent;
    and on one thread."""
    import numpy as np

    import oracle
    cpu = host_cpu()
    threads = max(1, min(16, cpu["nproc"]))
    t0 = time.perf_counter()
    S = oracle.Scene(scene)
    build_s = time.perf_counter() - t0
    npix = W * H

    def run(nthreads, budget, chunk):
        done, frame = 0, 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget and frame < 1000:
            first = done % npix
            px = np.arange(first, min(npix, first + chunk), dtype=np.int32)
            S.render(cam, pixels=px, spp=SPP, max_depth=DEPTH, seed=0, frame=frame, rr_start=RR, threads=nthreads)
            done += px.size
            if done % npix == 0:
                frame += 1
        return done, frame, time.perf_counter() - t0

    done, frame, dt = run(threads, budget_s, 262144)
    done1, _, dt1 = run(1, single_s, 16384)
    return {"value": done * SPP / dt, "unit": "path-samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} paths = {done / npix:.2f} frames of the {W}x{H} 1-spp workload (frames 0..{frame}), "
                      f"{dt:.1f} s render on {threads} threads, BVH build {build_s:.1f} s excluded",
            "host": cpu,
            "threads_note": "threads = the CPUs this process may use, capped at 16 (the host share of one GPU)",
            "single_thread": {"value": done1 * SPP / dt1, "sample": f"first {done1} paths of frame 0, {dt1:.1f} s"}}


def copy_ceiling(torch):
    """Measured device-to-device copy bandwidth (1 GiB read + 1 GiB written
    per copy): the HBM ceiling the streaming stages can reach."""
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / 5
    del a, b
    return {"value": 2 * (1 << 30) / dt / 1e9, "unit": "GB/s", "bytes_per_copy": 2 * (1 << 30)}


def time_frames(torch, R, img, k, first, in_flight, **kw):
    """Seconds for k frames (first .. first + k - 1), frame by frame or with
    three in flight, after the caller's warm-up."""
    torch.cuda.synchronize()
    t = time.perf_counter()
    if in_flight:
        R.render_frames(k, out=img, frame=first, **kw)
    else:
        for i in range(k):
            R.render(out=img, frame=first + i, **kw)
    torch.cuda.synchronize()
    return time.perf_counter() - t


# set by --serial-stages: wavefront frames rendered one by one run every
# stage on the render stream (no shadow stage beside the extend stage)
SERIAL_FLAGS = 0


def schedule_run(torch, R, img, params, steps, warmup, kw, mode):
    """Frame-by-frame and in-flight rates of one schedule."""
    out = {"params": params}
    for name, infl in [("frame_by_frame", False), ("frames_in_flight", True)]:
        p = params[name]
        if not infl and mode == "wave" and SERIAL_FLAGS:
            p = dict(p, flags=p.get("flags", 0) | SERIAL_FLAGS)
        time_frames(torch, R, img, max(1, warmup), 0, infl, mode=mode, **kw, **p)
        dt = time_frames(torch, R, img, steps, warmup, infl, mode=mode, **kw, **p)
        out[name] = {"ms_per_step": dt * 1e3 / steps, "value": W * H * SPP * steps / dt}
    return out


def profiled_frames(R, img, ptmi, mode, params, k, first, kw):
    """k frames with per-stage HIP-event timing, then the same k frames with
    the work-counting kernels: stage times, launches, items, algorithmic
    state bytes, rays, node visits and triangle tests (summed).  Wavefront
    stages run one after another (PT_FLAG_SERIAL_STAGES), so that each
    kernel's event time is its own."""
    acc = {"stage_ms": {}, "launches": {}, "items": {}, "bytes": {}, "node_visits": {}, "tri_tests": {},
           "extension_rays": 0, "shadow_rays": 0, "frames": k}
    serial = ptmi.FLAG_SERIAL_STAGES if mode == "wave" else 0
    for flag, keys in [(ptmi.FLAG_PROFILE, ("stage_ms", "launches", "items", "bytes")),
                       (ptmi.FLAG_COUNT_WORK, ("node_visits", "tri_tests"))]:
        for i in range(k):
            p = dict(params)
            p["flags"] = p.get("flags", 0) | flag | serial
            R.render(out=img, mode=mode, frame=first + i, **kw, **p)
            st = R.stats()
            for key in keys:
                for s, v in st[key].items():
                    acc[key][s] = acc[key].get(s, 0) + v
            if flag == ptmi.FLAG_PROFILE:
                acc["extension_rays"] += st["extension_rays"]
                acc["shadow_rays"] += st["shadow_rays"]
    return acc


def roofline_entry(kernel, launches, ms, state_bytes, nodes, tris, prof, copy_gbs):
    """Roofline figures of one kernel from its summed event times, launches,
    algorithmic state bytes and traversal work, with the measured HBM
    traffic and counters of the committed profile (None when stale)."""
    avg_ms = ms / launches
    e = {"kernel": kernel, "launches": launches, "avg_launch_ms": avg_ms}
    per_bytes = state_bytes / launches
    gbs = per_bytes / (avg_ms * 1e-3) / 1e9
    e["state"] = {"bytes_per_launch": per_bytes, "achieved_gbs": gbs, "frac_hbm_peak": gbs / HBM_PEAK_GBS,
                  "frac_copy_ceiling": gbs / copy_gbs if copy_gbs else None}
    if nodes is not None:
        per_flops = (FLOPS_PER_NODE * nodes + FLOPS_PER_TRI * tris) / launches
        tf = per_flops / (avg_ms * 1e-3) / 1e12
        e["alu"] = {"flops_per_launch": per_flops, "node_visits_per_launch": nodes / launches,
                    "tri_tests_per_launch": tris / launches, "achieved_tflops": tf,
                    "frac_fp32_peak": tf / FP32_PEAK_TFLOPS, "frac_fp32_packed_peak": tf / FP32_PEAK_PACKED_TFLOPS}
    k = (prof or {}).get("kernels", {}).get(kernel)
    if k:
        traffic = k.get("hbm_bytes_per_dispatch")
        e["measured"] = {"hbm_bytes_per_dispatch": traffic,
                         "hbm_gbs": traffic / (avg_ms * 1e-3) / 1e9 if traffic else None,
                         "traffic_over_state": traffic / per_bytes if traffic and per_bytes else None,
                         "profile_avg_us": k.get("avg_us"), "valu_per_cu_cycle": k.get("valu_per_cu_cycle"),
                         "l2_hit_rate": k.get("l2_hit_rate"), "waves_per_simd": k.get("waves_per_simd"),
                         "vgpr": k.get("vgpr"), "lds": k.get("lds"), "scratch": k.get("scratch")}
    return e


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--serial-stages", action="store_true",
                    help="wavefront frames rendered one by one run every stage on the render stream (profiled runs "
                         "take this, so that the profile's kernel times match the rooflines' per-kernel ones)")
    ap.add_argument("--adjoint-replay", default="mega,wave,keep",
                    help="comma-separated schedules of the adjoint's radiance replay: mega, wave, and keep (each "
                         "also keeping the intersections for the gradient replay); profiled runs take mega,keep "
                         "only, so that the wavefront kernels' averages are the forward frame's")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the divergence and batched workload summaries and the compaction ablation")
    ap.add_argument("--schedules", default="wave_hybrid,wave_pure,mega",
                    help="comma-separated schedules to run: wave_hybrid, wave_pure, mega")
    ap.add_argument("--no-tune", action="store_true", help="default launch parameters instead of the autotuner")
    ap.add_argument("--fixed", action="store_true",
                    help="launch parameters the autotuner chose on MI355X for this workload, without tuning "
                         "(for profiled runs)")
    ap.add_argument("--params", default=None,
                    help='launch parameters as JSON, e.g. {"wave": {"block": 256, "grid_mult": 8}} (no tuning)')
    ap.add_argument("--batch", action="store_true",
                    help="batched workload instead: 64 jobs, 10k-2M triangles each, mixed resolutions and spp")
    ap.add_argument("--divergence", action="store_true",
                    help="divergence workload instead: ~10M triangles, 64 material ids, 4 spp, depth 16")
    ap.add_argument("--max-leaf", type=int, default=0, help="triangles per BVH leaf, 1..8 (0 = library default, 1)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device-to-device copy (calibrates the HBM byte counters)")
    args = ap.parse_args()
    global SERIAL_FLAGS
    if args.copy_probe:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 4, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU sharding is a design "
              f"note, not a measured configuration", file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    from paper_2605_27323_amd import autotune, profiles, ptmi, scenes
    if args.serial_stages:
        SERIAL_FLAGS = ptmi.FLAG_SERIAL_STAGES

    if args.batch:
        print(json.dumps(batch_bench(args, torch, ptmi, scenes, autotune)), flush=True)
        return
    if args.divergence:
        print(json.dumps(divergence_bench(args, torch, ptmi, scenes)), flush=True)
        return
    t0 = time.perf_counter()
    scene, cam = scenes.procedural(seed=2, n_objects=2000, width=W, height=H)
    nt = scene["indices"].shape[0]
    R = ptmi.Renderer(scene, cam, max_leaf=args.max_leaf)
    log(f"scene {nt} triangles, BVH {R.info.node_count} nodes depth {R.info.depth}, "
        f"built in {R.info.build_seconds:.2f} s (setup {time.perf_counter() - t0:.1f} s)")
    kw = dict(spp=SPP, max_depth=DEPTH, rr_start=RR, nee=True, seed=0)
    img = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    schedules = [x for x in args.schedules.split(",") if x]
    if not schedules or any(x not in ("wave_hybrid", "wave_pure", "mega") for x in schedules):
        raise SystemExit(f"unknown schedule list {args.schedules!r}")
    modes = (["wave"] if any(x.startswith("wave") for x in schedules) else []) + (["mega"] if "mega" in schedules else [])

    # launch parameters per schedule, frame by frame and with frames in flight
    tuned = {}
    for mode in modes:
        if args.params:
            given = json.loads(args.params)
            p = dict(given.get(mode, FIXED_PARAMS[mode]))
            tuned[mode] = {"frame_by_frame": p, "frames_in_flight": p}
        elif args.fixed:
            tuned[mode] = {"frame_by_frame": dict(FIXED_PARAMS[mode]), "frames_in_flight": dict(FIXED_PARAMS[mode])}
        elif args.no_tune:
            tuned[mode] = {"frame_by_frame": {}, "frames_in_flight": {}}
        else:
            tuned[mode] = {}
            for name, infl in [("frame_by_frame", False), ("frames_in_flight", True)]:
                t = time.perf_counter()
                tuned[mode][name] = autotune.tune_frame(R, mode=mode, cache=None, log=log, in_flight=infl, **kw)
                log(f"autotune {mode} {name}: {tuned[mode][name]} ({time.perf_counter() - t:.1f} s)")

    sched = {}
    if "wave_hybrid" in schedules:
        sched["wave_hybrid"] = schedule_run(torch, R, img, tuned["wave"], args.steps, args.warmup, kw, "wave")
    if "wave_pure" in schedules:
        pure = {n: dict(p, **PURE) for n, p in tuned["wave"].items()}
        sched["wave_pure"] = schedule_run(torch, R, img, pure, args.steps, args.warmup, kw, "wave")
    if "mega" in modes:
        sched["mega"] = schedule_run(torch, R, img, tuned["mega"], args.steps, args.warmup, kw, "mega")
    for s, v in sched.items():
        log(f"{s}: {v['frame_by_frame']['ms_per_step']:.3f} ms/frame, in flight "
            f"{v['frames_in_flight']['ms_per_step']:.3f} ms/frame")

    copy = copy_ceiling(torch)
    copy_gbs = copy["value"]
    prof = profiles.load(PROFILE)
    out_roof = {}
    frame_stage_ms = {}
    wave_sum = {}
    k = min(args.steps, 16)
    if "wave" in modes:
        # stage profile at the fixed launch parameters (those of the committed
        # rocprofv3 profiles), frame by frame on the render stream
        for name, params in [("hybrid", FIXED_PARAMS["wave"]), ("pure", dict(FIXED_PARAMS["wave"], **PURE))]:
            if f"wave_{name}" not in schedules:
                continue
            acc = profiled_frames(R, img, ptmi, "wave", params, k, args.warmup, kw)
            frame_stage_ms[name] = {s: v / k for s, v in acc["stage_ms"].items()}
            log(f"wavefront ({name}) stage ms/frame: " +
                ", ".join(f"{s} {v:.3f}" for s, v in frame_stage_ms[name].items()))
            lds = params.get("stack_lds", 8)
            kname = {"extend": f"ptmi::k_extend<{lds}, false, false>", "shadow": f"ptmi::k_shadow<{lds}, false, false>",
                     "tail": f"ptmi::k_shade_tail<{lds}, false, false, false>", "shade": "ptmi::k_shade<false, false>"}
            for st in ["extend", "shadow", "shade", "tail"]:
                if st not in acc["launches"]:
                    continue
                trav = st in ("extend", "shadow", "tail")
                out_roof[f"{st}_{name}"] = roofline_entry(
                    kname[st], acc["launches"][st], acc["stage_ms"][st], acc["bytes"].get(st, 0.0),
                    acc["node_visits"].get(st, 0) if trav else None, acc["tri_tests"].get(st, 0) if trav else None,
                    prof if name == "hybrid" else None, copy_gbs)
            wave_sum[name] = {
                "rays": {"extension": acc["extension_rays"] / k, "shadow": acc["shadow_rays"] / k},
                "dominant": max(acc["stage_ms"], key=acc["stage_ms"].get),
                "share": {s: v / sum(acc["stage_ms"].values()) for s, v in acc["stage_ms"].items()},
                "items": {s: v / k for s, v in acc["items"].items()},
                "nodes": {s: v / k for s, v in acc["node_visits"].items()},
                "tris": {s: v / k for s, v in acc["tri_tests"].items()},
                "state_bytes": sum(acc["bytes"].values()) / k}
    if "mega" in modes:
        acc = profiled_frames(R, img, ptmi, "mega", FIXED_PARAMS["mega"], k, args.warmup, kw)
        waves = FIXED_PARAMS["mega"].get("mega_waves", 4)
        out_roof["mega"] = roofline_entry(
            f"ptmi::k_mega<{FIXED_PARAMS['mega']['stack_lds']}, false, {waves}, false, false>", acc["launches"]["mega"],
            acc["stage_ms"]["mega"], acc["bytes"]["mega"], acc["node_visits"]["mega"], acc["tri_tests"]["mega"],
            prof, copy_gbs)

    out_adj = None
    if not args.no_adjoint:
        out_adj = adjoint_bench(ptmi, scene, torch, args, prof, copy_gbs, out_roof)

    head = "wave_hybrid" if "wave_hybrid" in sched else ("wave_pure" if "wave_pure" in sched else "mega")
    hv = sched[head]["frames_in_flight"]
    roofline = None
    hname = {"wave_hybrid": "hybrid", "wave_pure": "pure"}.get(head)
    ws = wave_sum.get(hname)
    rays = ws["rays"] if ws else None
    if ws and f"extend_{hname}" in out_roof:
        # the dominant kernel of the headline frame: the extension rays'
        # traversal, against the HBM peak on its algorithmic state bytes
        # (48 B per ray: read the ray, write the hit)
        r = out_roof[f"extend_{hname}"]
        roofline = {"bound": "hbm", "achieved": r["state"]["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": r["state"]["frac_hbm_peak"],
                    "traffic": (r.get("measured") or {}).get("hbm_bytes_per_dispatch"),
                    "kernel": r["kernel"], "avg_launch_ms": r["avg_launch_ms"],
                    "launches_per_frame": r["launches"] / k, "bytes_per_launch": r["state"]["bytes_per_launch"],
                    "frac_copy_ceiling": r["state"]["frac_copy_ceiling"], "alu": r.get("alu"),
                    "measured": r.get("measured"), "stage_share": ws["share"].get("extend"),
                    "dominant_stage": ws["dominant"],
                    "launch_params": dict(FIXED_PARAMS["wave"], **(PURE if hname == "pure" else {}))}
    # frames the library keeps in flight: its frames workspace in frame slots
    # (one wavefront workspace and one image each, 256-byte aligned)
    import ctypes
    a0 = R.args(mode="wave", spp=SPP, max_depth=DEPTH)
    n1, nf = ctypes.c_uint64(), ctypes.c_uint64()
    ptmi.lib().pt_workspace_size(R.h, ctypes.byref(a0), ctypes.byref(n1))
    ptmi.lib().pt_frames_workspace_size(R.h, ctypes.byref(a0), ctypes.byref(nf))
    in_flight = int(nf.value // (((n1.value + 12 * W * H) + 255) // 256 * 256))
    out = {
        "metric": "path samples/s wavefront vs megakernel @1080p, 1M tris; adjoint samples/s",
        "value": hv["value"],
        "unit": "path-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hv["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"procedural scene {nt} triangles (1000 icospheres + 1000 tessellated boxes, "
                               f"ground, 16 quad lights), {W}x{H}, {SPP} spp/frame, max depth {DEPTH}, "
                               f"roulette from {RR}, light sampling on; "
                               + ({"wave_pure": "pure wavefront schedule (separate extend / shade / shadow "
                                               "launches over compacted queues at every bounce)",
                                  "mega": "megakernel"}.get(head) or "wavefront schedule with the hybrid tail (separate extend / shade / shadow "
                                  "launches over compacted queues while they are long, the paths still live at "
                                  "the tail bounce finished megakernel-style in one launch)"
                                  ) +
                               f", progressive frames with {in_flight} in flight (bit-identical to frame by frame)",
                   "width": W, "height": H, "spp": SPP, "max_depth": DEPTH, "triangles": nt,
                   "frames_in_flight": in_flight},
        "schedules": sched,
        "wave_over_mega": ({s: {n: sched["mega"][n]["ms_per_step"] / sched[s][n]["ms_per_step"]
                                for n in ("frame_by_frame", "frames_in_flight")}
                            for s in ("wave_pure", "wave_hybrid") if s in sched} if "mega" in sched else None),
        "rays_per_s": ((rays["extension"] + rays["shadow"]) / (hv["ms_per_step"] * 1e-3)) if rays else None,
        "rays_per_frame": rays,
        "stage_ms_per_frame": frame_stage_ms,
        "roofline": roofline,
        "rooflines": out_roof,
        "state_traffic": ({"bytes_per_frame": ws["state_bytes"],
                           "frac_hbm_peak_at_headline": ws["state_bytes"] / (hv["ms_per_step"] * 1e-3) / 1e9 /
                           HBM_PEAK_GBS} if ws else None),
        "wavefront_work_per_frame": {n: {"items": v["items"], "node_visits": v["nodes"], "tri_tests": v["tris"],
                                         "rays": v["rays"], "stage_share": v["share"]} for n, v in wave_sum.items()},
        "hbm_copy_ceiling": copy,
        "profile": {"name": PROFILE, "current": prof is not None},
        "paper_context": "paper reports ~16% (1.138x by its table) wavefront over megakernel on an RTX 3060 Ti "
                         "with RT cores, A Beautiful Game scene",
    }
    if out_adj:
        out["adjoint"] = out_adj
    if not args.no_extra and "wave" in modes:
        out["compaction"] = compaction_bench(torch, R, img, ptmi, kw, tuned["wave"]["frame_by_frame"])
    if not args.no_extra:
        del R
        torch.cuda.empty_cache()
        out["instancing"] = instancing_bench(args, torch, ptmi, scenes)
        torch.cuda.empty_cache()
        out["attributes"] = attributes_bench(args, torch, ptmi, scenes)
        torch.cuda.empty_cache()
        out["divergence"] = divergence_bench(args, torch, ptmi, scenes, frames=2, summary=True)
        torch.cuda.empty_cache()
        out["batch"] = batch_bench(args, torch, ptmi, scenes, None, runs=2, summary=True)
    if not args.no_cpu:
        log("oracle CPU baseline ...")
        out["cpu_baseline"] = cpu_baseline(scene, cam)
    print(json.dumps(out), flush=True)


def compaction_bench(torch, R, img, ptmi, kw, params, k=6):
    """Pure wavefront with compaction (live paths packed into the next queue
    after every bounce) against no compaction (every path slot dispatched
    every bounce, finished ones skipped), at depth 8 and 16 (paper Sec. 3.1:
    the gain grows with the maximum depth); and the paper's two-slot live
    count with a promote kernel after every bounce against one counter per
    bounce."""
    res = {}
    base = dict(params, **PURE)
    base.pop("flags", None)
    for depth in (DEPTH, 16):
        r = {}
        for name, flags in [("compacted", 0), ("no_compaction", ptmi.FLAG_NO_COMPACT),
                            ("two_slot_promote", ptmi.FLAG_TWO_SLOT)]:
            p = dict(base, flags=flags)
            a = dict(kw, max_depth=depth)
            time_frames(torch, R, img, 1, 0, False, mode="wave", **a, **p)
            dt = time_frames(torch, R, img, k, 1, False, mode="wave", **a, **p)
            r[name] = {"ms_per_frame": dt * 1e3 / k}
        r["gain"] = r["no_compaction"]["ms_per_frame"] / r["compacted"]["ms_per_frame"]
        r["two_slot_over_per_bounce"] = r["two_slot_promote"]["ms_per_frame"] / r["compacted"]["ms_per_frame"]
        res[f"depth{depth}"] = r
        log(f"compaction depth {depth}: {r['compacted']['ms_per_frame']:.3f} ms vs "
            f"{r['no_compaction']['ms_per_frame']:.3f} ms without ({r['gain']:.2f}x)")
    return res


def instancing_bench(args, torch, ptmi, scenes, k=8):
    """Two-level scene (4016 instances of 34 shared meshes, ~1M instanced
    triangles, the procedural scene's layout) against its flattened copy:
    device bytes of the acceleration structure and triangles, and ms per
    frame of the hybrid wavefront and the megakernel, frame by frame."""
    sc, inst, cam = scenes.instanced_procedural(seed=6, width=W, height=H)
    flat = scenes.flatten_instances(sc, inst)
    kw = dict(spp=SPP, max_depth=DEPTH, rr_start=RR, nee=True, seed=0)
    img = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    res = {}
    for name, R in [("instanced", ptmi.Renderer(sc, cam, instances=inst)), ("flattened", ptmi.Renderer(flat, cam))]:
        i = R.info
        r = {"triangles": R.nt, "instances": i.instance_count, "node_bytes": i.node_bytes, "tri_bytes": i.tri_bytes,
             "instance_bytes": i.instance_bytes, "build_s": i.build_seconds,
             "device_bytes": i.node_bytes + i.tri_bytes + i.instance_bytes + i.light_bytes}
        for mode, p in [("wave_hybrid", dict(FIXED_PARAMS["wave"], mode="wave")),
                        ("mega", dict(FIXED_PARAMS["mega"], mode="mega"))]:
            time_frames(torch, R, img, 2, 0, False, **kw, **p)
            r[f"{mode}_ms_per_frame"] = time_frames(torch, R, img, k, 2, False, **kw, **p) * 1e3 / k
        res[name] = r
        log(f"{name}: {r}")
        del R
    res["memory_ratio"] = res["flattened"]["device_bytes"] / res["instanced"]["device_bytes"]
    res["time_ratio_wave"] = res["instanced"]["wave_hybrid_ms_per_frame"] / res["flattened"]["wave_hybrid_ms_per_frame"]
    res["workload"] = (f"{len(inst['inst_mesh'])} instances of {len(inst['mesh_first'])} meshes "
                       f"({sc['indices'].shape[0]} unique triangles), {W}x{H}, {SPP} spp, depth {DEPTH}, roulette "
                       f"from {RR}; flattened = every instance's triangles in world space")
    return res


def attributes_bench(args, torch, ptmi, scenes, k=8):
    """The benchmark geometry with shading attributes (smooth-shaded
    icospheres, checker textures, half of the conductors coated) against the
    same geometry without them: attribute bytes and ms per frame of the
    hybrid wavefront and the megakernel, frame by frame."""
    kw = dict(spp=SPP, max_depth=DEPTH, rr_start=RR, nee=True, seed=0)
    img = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    res = {}
    for name, attr in [("attributes", True), ("plain", False)]:
        scene, cam = scenes.procedural(seed=2, n_objects=2000, width=W, height=H, attributes=attr)
        R = ptmi.Renderer(scene, cam, max_leaf=args.max_leaf)
        r = {"attribute_bytes": R.info.attribute_bytes,
             "coated_materials": int((scene["materials"][:, 0] == scenes.COATED).sum()),
             "textured_materials": int((scene["materials"][:, 3] > 0).sum())}
        for mode, p in [("wave_hybrid", dict(FIXED_PARAMS["wave"], mode="wave")),
                        ("mega", dict(FIXED_PARAMS["mega"], mode="mega"))]:
            time_frames(torch, R, img, 2, 0, False, **kw, **p)
            r[f"{mode}_ms_per_frame"] = time_frames(torch, R, img, k, 2, False, **kw, **p) * 1e3 / k
        res[name] = r
        log(f"{name}: {r}")
        del R
    res["time_ratio_wave"] = res["attributes"]["wave_hybrid_ms_per_frame"] / res["plain"]["wave_hybrid_ms_per_frame"]
    res["time_ratio_mega"] = res["attributes"]["mega_ms_per_frame"] / res["plain"]["mega_ms_per_frame"]
    res["workload"] = (f"procedural scene (1019958 triangles) with and without shading attributes, {W}x{H}, {SPP} "
                       f"spp, depth {DEPTH}, roulette from {RR}")
    return res


def batch_bench(args, torch, ptmi, scenes, autotune, runs=None, summary=False):
    """64 jobs: per job a procedural scene of T triangles (T log-uniform in
    [1e4, 2e6]), a resolution from {256^2, 512^2, 1024^2, 1920x1080}, 1..8
    spp, depth 8, roulette from 3; all in one batched persistent wavefront."""
    import numpy as np
    t0 = time.perf_counter()
    specs = scenes.batch_jobs(seed=4, n_jobs=64)
    Rs, job_args = [], []
    ntri = 0
    for j, sp in enumerate(specs):
        sc, cam = scenes.procedural(seed=sp["scene_seed"], n_objects=sp["n_objects"], width=sp["width"],
                                    height=sp["height"])
        Rs.append(ptmi.Renderer(sc, cam, max_leaf=args.max_leaf))
        ntri += sc["indices"].shape[0]
        job_args.append(dict(spp=sp["spp"], max_depth=DEPTH, rr_start=RR, nee=True, seed=0, job=j))
    total = sum(R.width * R.height * a["spp"] for R, a in zip(Rs, job_args))
    log(f"batch: {len(Rs)} jobs, {ntri} triangles, {total} path samples (setup {time.perf_counter() - t0:.1f} s)")
    if autotune is not None and not args.no_tune and not args.fixed:
        opts = autotune.tune_batch(Rs, job_args, cache=None, log=log)
    else:
        opts = dict(BATCH_OPTS)
    log(f"batch options {opts}")
    _, _, r = ptmi.render_batch(Rs, job_args, **opts)
    ws = r["workspace"]
    res = []
    for _ in range(runs or max(1, args.steps // 16)):
        _, ms, r = ptmi.render_batch(Rs, job_args, workspace=ws, **opts)
        res.append((r["seconds"], ms, r))
    sec = min(t for t, _, _ in res)
    ms, r = [(m, rr) for t, m, rr in res if t == sec][0]
    lat = {"p50": float(np.percentile(ms, 50)), "p99": float(np.percentile(ms, 99)), "max": float(np.max(ms))}
    log(f"batch: {sec * 1e3:.1f} ms, {total / sec / 1e6:.1f} M path-samples/s, latency {lat}")
    body = {"value": total / sec, "unit": "path-samples/s", "ms": sec * 1e3, "job_latency_ms": lat,
            "iterations": r["iterations"], "graph_launches": r["launches"], "batch_options": opts,
            "runs": len(res), "triangles": ntri, "path_samples": total,
            "workload": f"64 jobs, {ntri} triangles in total, {total} path samples, depth {DEPTH}, roulette from "
                        f"{RR}, batched persistent wavefront with a hipGraph loop"}
    if summary:
        return body
    return {"metric": "batched path samples/s (64 jobs)", "value": total / sec, "unit": "path-samples/s",
            "n_gpus": 1, "steps": len(res), "warmup": 1, "ms_per_step": sec * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": body["workload"], "triangles": ntri, "path_samples": total},
            "job_latency_ms": lat, "iterations": r["iterations"], "graph_launches": r["launches"],
            "batch_options": opts}


def divergence_bench(args, torch, ptmi, scenes, frames=None, summary=False):
    """~10M triangles, 64 material ids (Lambertian, conductor, rough
    dielectric, emissive), 1920x1080, 4 spp, depth 16, roulette from 3:
    megakernel, wavefront (hybrid and pure), wavefront with the material
    sort and with the ray sort, and the hybrid wavefront and the megakernel
    with frames in flight."""
    t0 = time.perf_counter()
    scene, cam = scenes.procedural(seed=3, n_objects=20000, width=W, height=H, material_mode="divergence")
    nt = scene["indices"].shape[0]
    R = ptmi.Renderer(scene, cam, max_leaf=args.max_leaf)
    log(f"divergence scene {nt} triangles, BVH depth {R.info.depth} (setup {time.perf_counter() - t0:.1f} s)")
    kw = dict(spp=4, max_depth=16, rr_start=3, nee=True, seed=0)
    img = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    res = {}
    k = frames or max(2, args.steps // 8)
    given = json.loads(args.params) if args.params else {}
    wave = dict(given.get("wave", DIVERGENCE_PARAMS["wave"]))
    mega = dict(given.get("mega", DIVERGENCE_PARAMS["mega"]))

    def sorted_by(flag):
        return dict(wave, mode="wave", flags=wave.get("flags", 0) | flag,
                    sort_threshold=wave.get("sort_threshold", 1 << 16))

    runs = [("mega", dict(mode="mega", **mega)), ("wave_hybrid", dict(mode="wave", **wave)),
            ("wave_pure", dict(dict(mode="wave", **wave), **PURE)),
            ("wave_hybrid_material_sort", sorted_by(ptmi.FLAG_SORT_MATERIAL)),
            ("wave_hybrid_ray_sort", sorted_by(ptmi.FLAG_SORT_RAYS))]
    for name, extra in runs:
        time_frames(torch, R, img, 1, 0, False, **kw, **extra)
        dt = time_frames(torch, R, img, k, 1, False, **kw, **extra) / k
        res[name] = {"ms_per_frame": dt * 1e3, "path_samples_per_s": W * H * 4 / dt}
        log(f"divergence {name}: {dt * 1e3:.2f} ms/frame")
    for name, extra in [("mega_in_flight", dict(mode="mega", **mega)),
                        ("wave_hybrid_in_flight", dict(mode="wave", **wave))]:
        time_frames(torch, R, img, 2, 0, True, **kw, **extra)
        dt = time_frames(torch, R, img, max(k, 3), 2, True, **kw, **extra) / max(k, 3)
        res[name] = {"ms_per_frame": dt * 1e3, "path_samples_per_s": W * H * 4 / dt}
        log(f"divergence {name}: {dt * 1e3:.2f} ms/frame")
    best = max((r for r in res if r.startswith("wave")), key=lambda r: res[r]["path_samples_per_s"])
    workload = f"procedural {nt} triangles, 64 material ids, {W}x{H}, 4 spp, depth 16, roulette from 3"
    if summary:
        return {"workload": workload, "frames_per_run": k, "schedules": res, "best_wavefront": best,
                "wave_over_mega_frame_by_frame": res["mega"]["ms_per_frame"] / res["wave_hybrid"]["ms_per_frame"],
                "launch_params": {"wave": wave, "mega": mega}}
    return {"metric": "path samples/s, divergence workload", "value": res[best]["path_samples_per_s"],
            "unit": "path-samples/s", "n_gpus": 1, "steps": k, "warmup": 1,
            "ms_per_step": res[best]["ms_per_frame"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{workload}; best wavefront schedule: {best}"}, "schedules": res}


def adjoint_bench(ptmi, scene, torch, args, prof, copy_gbs, roof):
    """Backward (path replay) of the 512x512, 8 spp, depth 6 frame: adjoint
    samples/s with replay A (each path's radiance) run two ways, as the
    megakernel-style kernel and as the wavefront stages (the same per-path
    radiance bit for bit), and the rooflines of the adjoint kernels (replay
    B adds the gradients).  The replays trace the rays of the forward
    megakernel frame with the same arguments, so their node visits and
    triangle tests are those of that frame."""
    cam = dict(eye=(0.0, 50.0, -130.0), target=(0.0, 40.0, 0.0), up=(0.0, 1.0, 0.0), vfov_deg=50.0,
               width=512, height=512)
    try:
        R = ptmi.Renderer(scene, cam, max_leaf=args.max_leaf)
        kw = dict(spp=8, max_depth=6, rr_start=-1, nee=True, seed=0)
        d_img = torch.ones((512, 512, 3), dtype=torch.float32, device="cuda")
        ga = torch.zeros_like(R.albedo)
        ge = torch.zeros_like(R.emission)
        k = max(4, args.steps // 8)
        n = 512 * 512 * 8 * k
        variants = {"replay_a_megakernel": dict(ADJOINT_PARAMS["mega"], mode="mega"),
                    "replay_a_wavefront": dict(ADJOINT_PARAMS["wave"], mode="wave"),
                    "replay_a_megakernel_keep_hits": dict(ADJOINT_PARAMS["mega"], mode="mega",
                                                          flags=ptmi.FLAG_KEEP_HITS),
                    "replay_a_wavefront_keep_hits": dict(ADJOINT_PARAMS["wave_keep"], mode="wave",
                                                         flags=ptmi.FLAG_KEEP_HITS)}
        pick = args.adjoint_replay.split(",")
        variants = {n: p for n, p in variants.items()
                    if p["mode"] in pick and (("keep" in pick) or not n.endswith("keep_hits"))}
        res = {}
        wave_stages = ("raygen", "extend", "shade", "shadow", "tail")
        for name, p in variants.items():
            fl = p.get("flags", 0)
            p = {x: v for x, v in p.items() if x != "flags"}
            R.backward(d_img, ga, ge, flags=fl, **kw, **p)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for i in range(k):
                R.backward(d_img, ga, ge, frame=i, flags=fl, **kw, **p)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            # per-kernel event times
            ms = {"replay_a": 0.0, "adjoint": 0.0}
            by = {"adjoint_radiance": 0.0, "adjoint": 0.0}
            for i in range(k):
                R.backward(d_img, ga, ge, frame=i, flags=ptmi.FLAG_PROFILE | fl, **kw, **p)
                st = R.stats()
                ms["adjoint"] += st["stage_ms"]["adjoint"]
                by["adjoint"] += st["bytes"]["adjoint"]
                if p["mode"] == "mega":
                    ms["replay_a"] += st["stage_ms"]["adjoint_radiance"]
                    by["adjoint_radiance"] += st["bytes"]["adjoint_radiance"]
                else:
                    ms["replay_a"] += sum(st["stage_ms"].get(x, 0.0) for x in wave_stages)
            res[name] = {"value": n / dt, "ms_per_backward": dt * 1e3 / k, "keep_hits": fl != 0,
                         "launch_params": {x: v for x, v in p.items() if x != "mode"},
                         "ms_per_kernel": {x: v / k for x, v in ms.items()}, "_ms": ms, "_by": by}
            log(f"adjoint ({name}): {dt * 1e3 / k:.3f} ms per backward, {n / dt / 1e6:.1f} M samples/s")
        nodes = tris = 0
        img = torch.empty((512, 512, 3), dtype=torch.float32, device="cuda")
        for i in range(k):
            R.render(out=img, mode="mega", frame=i, flags=ptmi.FLAG_COUNT_WORK, **kw)
            st = R.stats()
            nodes += st["node_visits"]["mega"]
            tris += st["tri_tests"]["mega"]
        if "replay_a_megakernel" in res:
            mg = res["replay_a_megakernel"]
            roof["adjoint_radiance"] = roofline_entry("ptmi::k_adjoint_radiance<8, false, false>", k,
                                                      mg["_ms"]["replay_a"], mg["_by"]["adjoint_radiance"], nodes, tris,
                                                      prof, copy_gbs)
        best = min(res, key=lambda x: res[x]["ms_per_backward"])
        # the gradient replay of the fastest variant; reading kept
        # intersections it traces nothing (no traversal work)
        kb = res[best]["keep_hits"]
        roof["adjoint"] = roofline_entry(f"ptmi::k_adjoint<8, false, {'true' if kb else 'false'}>", k,
                                         res[best]["_ms"]["adjoint"], res[best]["_by"]["adjoint"],
                                         None if kb else nodes, None if kb else tris, prof, copy_gbs)
        for r in res.values():
            r.pop("_ms")
            r.pop("_by")
        return {"value": res[best]["value"], "unit": "adjoint samples/s",
                "ms_per_backward": res[best]["ms_per_backward"], "best": best, "variants": res,
                "ms_per_kernel": res[best]["ms_per_kernel"],
                "config": "same scene, 512x512, 8 spp, max depth 6, roulette off"}
    except ptmi.PtError as e:
        log(f"adjoint unavailable: {e}")
        return None


if __name__ == "__main__":
    main()
