#!/usr/bin/env python3
"""Benchmark: path samples/s of the wavefront and the megakernel on the
procedural ~1M-triangle scene at 1920x1080, 1 spp per frame, max depth 8,
Russian roulette from vertex 3, next-event estimation on; plus the adjoint
(path-replay backward) samples/s on the same scene at 512x512, 8 spp,
depth 6, roulette off.

One step = one frame of the wavefront pipeline (raygen, extend, shade,
shadow, accumulate over all bounces).  Inputs are resident in device memory
before timing starts.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
# algorithmic flops of one BVH4 node visit (four slab tests of 26 flops:
# 6 subtractions, 6 multiplications, 12 min/max, slack multiply, compare)
# and of one watertight triangle test (51 flops on its full path)
FLOPS_PER_NODE = 104
FLOPS_PER_TRI = 51
# autotuner result on MI355X for the 1M-triangle 1080p workload
FIXED_PARAMS = {"wave": {"block": 256, "grid_mult": 8, "stack_lds": 8, "tail_threshold": 1 << 18, "tail_bounce": 4},
                "mega": {"block": 256, "grid_mult": 4, "stack_lds": 8}}
# launch parameters of the divergence workload (4 spp, depth 16)
DIVERGENCE_PARAMS = {"wave": {"block": 256, "grid_mult": 8, "stack_lds": 8, "tail_threshold": 1 << 18, "tail_bounce": 6},
                     "mega": {"block": 256, "grid_mult": 4, "stack_lds": 8}}
W, H, SPP, DEPTH, RR = 1920, 1080, 1, 8, 3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel, field="hbm_bytes_per_dispatch"):
    """HBM bytes per dispatch of `kernel` (or another recorded field) from the
    committed rocprofv3 counter summary, or None when the kernel sources
    changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_extend_procedural1M_1080p.json")
    if not os.path.exists(path):
        return None
    prof = json.load(open(path))
    h = hashlib.sha256()
    for f in ["device.h", "wavefront.h", "wave.h", "kernels.hip", "kernels.h", "ptmi_internal.h"]:
        h.update(open(os.path.join(ROOT, "paper_2605_27323_amd", "csrc", f), "rb").read())
    if h.hexdigest()[:16] != prof["source_hash"]:
        return None
    k = prof["kernels"].get(kernel)
    return k.get(field) if k else None


def cpu_baseline(scene, cam, budget_s=12.0, single_s=3.0):
    """The oracle (plain C, all host threads) on whole frames 0, 1, 2, ...
    of the benchmark workload, split in 262144-pixel chunks, until the time
    budget is spent."""
    import numpy as np

    import oracle
    # the cores this process may use, at most 16 (the host share of one GPU)
    threads = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()))
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--mode", default="both", choices=["both", "wave", "mega"])
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

    import numpy as np
    import torch

    from paper_2605_27323_amd import autotune, ptmi, scenes

    if args.batch:
        return batch_bench(args)
    if args.divergence:
        return divergence_bench(args)
    t0 = time.perf_counter()
    scene, cam = scenes.procedural(seed=2, n_objects=2000, width=W, height=H)
    nt = scene["indices"].shape[0]
    R = ptmi.Renderer(scene, cam, max_leaf=args.max_leaf)
    log(f"scene {nt} triangles, BVH {R.info.node_count} nodes depth {R.info.depth}, "
        f"built in {R.info.build_seconds:.2f} s (setup {time.perf_counter() - t0:.1f} s)")
    kw = dict(spp=SPP, max_depth=DEPTH, rr_start=RR, nee=True, seed=0)
    img = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    modes = ["wave", "mega"] if args.mode == "both" else [args.mode]
    tuned = {m: {} for m in modes}
    if args.params:
        given = json.loads(args.params)
        tuned = {m: dict(given.get(m, FIXED_PARAMS[m])) for m in modes}
    elif args.fixed:
        tuned = {m: dict(FIXED_PARAMS[m]) for m in modes}
    elif not args.no_tune:
        for mode in modes:
            t = time.perf_counter()
            tuned[mode] = autotune.tune_frame(R, mode=mode, cache=None, log=log, **kw)
            log(f"autotune {mode}: {tuned[mode]} ({time.perf_counter() - t:.1f} s)")

    def run(mode, k, first, flags=0):
        p = dict(tuned[mode])
        p["flags"] = p.get("flags", 0) | flags
        for i in range(k):
            R.render(out=img, mode=mode, frame=first + i, **kw, **p)

    res = {}
    for mode in modes:
        run(mode, args.warmup, 0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        run(mode, args.steps, args.warmup)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        res[mode] = dict(seconds=dt, ms=dt * 1e3 / args.steps, value=W * H * SPP * args.steps / dt)
        log(f"{mode}: {res[mode]['ms']:.3f} ms/frame, {res[mode]['value'] / 1e6:.1f} M path-samples/s")
    # the same frames with three in flight (pt_render_frames): one frame's
    # last, short bounces overlap the next frame's first ones
    inflight = {}
    tuned_inflight = {m: dict(tuned[m]) for m in modes}
    if not args.fixed and not args.no_tune and not args.params:
        for mode in modes:
            t = time.perf_counter()
            tuned_inflight[mode] = autotune.tune_frame(R, mode=mode, cache=None, log=log, in_flight=True, **kw)
            log(f"autotune {mode}, three frames in flight: {tuned_inflight[mode]} ({time.perf_counter() - t:.1f} s)")
    for mode in modes:
        p = dict(tuned_inflight[mode])
        R.render_frames(args.warmup, out=img, mode=mode, frame=0, **kw, **p)
        torch.cuda.synchronize()
        t = time.perf_counter()
        R.render_frames(args.steps, out=img, mode=mode, frame=args.warmup, **kw, **p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        inflight[mode] = dict(ms_per_step=dt * 1e3 / args.steps, value=W * H * SPP * args.steps / dt)
        log(f"{mode}, three frames in flight: {inflight[mode]['ms_per_step']:.3f} ms/frame, "
            f"{inflight[mode]['value'] / 1e6:.1f} M path-samples/s")

    stage_ms, launches, items, nbytes, nodes, tris = {}, {}, {}, {}, {}, {}
    rays = [0, 0]
    roofline, state_floor, frame_stage_ms = None, None, {}
    ext_rays_per_frame = sh_rays_per_frame = 0.0
    # stage profile and work counts at the fixed launch parameters, the ones
    # the committed rocprofv3 profiles were taken with (bench.py --fixed), so
    # that the roofline's mean launch time is comparable with them
    prof_params = dict(tuned["wave"]) if (args.params and "wave" in tuned) else dict(FIXED_PARAMS["wave"])

    def run_prof(first, flags):
        p = dict(prof_params)
        p["flags"] = p.get("flags", 0) | flags
        R.render(out=img, mode="wave", frame=first, **kw, **p)

    if "wave" in modes:
        # per-stage times with HIP events on the render stream, over the same
        # number of frames, plus ray counts, work items and algorithmic bytes
        for i in range(args.steps):
            run_prof(args.warmup + i, ptmi.FLAG_PROFILE)
            st = R.stats()
            for k, v in st["stage_ms"].items():
                stage_ms[k] = stage_ms.get(k, 0.0) + v
                launches[k] = launches.get(k, 0) + st["launches"][k]
            for k, v in st["items"].items():
                items[k] = items.get(k, 0) + v
                nbytes[k] = nbytes.get(k, 0.0) + st["bytes"][k]
            rays[0] += st["extension_rays"]
            rays[1] += st["shadow_rays"]
        # the same frames again with the work-counting kernels (node visits and
        # triangle tests; a separate, slower build, so not timed)
        for i in range(args.steps):
            run_prof(args.warmup + i, ptmi.FLAG_COUNT_WORK)
            st = R.stats()
            for k, v in st["node_visits"].items():
                nodes[k] = nodes.get(k, 0) + v
            for k, v in st["tri_tests"].items():
                tris[k] = tris.get(k, 0) + v
        frame_stage_ms = {k: v / args.steps for k, v in stage_ms.items()}
        log("wavefront stage ms/frame: " + ", ".join(f"{k} {v:.3f}" for k, v in frame_stage_ms.items()))
        ext_rays_per_frame = rays[0] / args.steps
        sh_rays_per_frame = rays[1] / args.steps
        # roofline of the stage kernel with the largest share of the frame.
        # Traversal kernels (extend, shadow, tail) are bound by vector ALU issue:
        # achieved = algorithmic flops per launch (FLOPS_PER_NODE per BVH node
        # visit, FLOPS_PER_TRI per triangle test, counted on the device) over the
        # mean launch time, against the fp32 vector peak.  The streaming stages
        # use their algorithmic path-state bytes against the HBM peak.
        dom = max(stage_ms, key=stage_ms.get)
        lds = prof_params.get("stack_lds", 16)
        kname = {"extend": f"ptmi::k_extend<{lds}, false>", "shade": "ptmi::k_shade",
                 "shadow": f"ptmi::k_shadow<{lds}, false>", "tail": f"ptmi::k_shade_tail<{lds}, false>",
                 "raygen": "ptmi::k_raygen", "accumulate": "ptmi::k_accumulate", "sort": "ptmi::k_sort_*"}[dom]
        dom_avg_ms = stage_ms[dom] / launches[dom]
        per_launch_bytes = nbytes.get(dom, 0.0) / launches[dom]
        state_gbs = per_launch_bytes / (dom_avg_ms * 1e-3) / 1e9
        common = {"kernel": kname, "traffic": measured_traffic(kname), "avg_launch_ms": dom_avg_ms,
                  "launches_per_frame": launches[dom] / args.steps, "items_per_frame": items.get(dom, 0) / args.steps,
                  "stage_share": stage_ms[dom] / sum(stage_ms.values()), "state_bytes_per_launch": per_launch_bytes,
                  "state_gbs": state_gbs, "launch_params": prof_params}
        if dom in ("extend", "shadow", "tail"):
            flops = FLOPS_PER_NODE * nodes.get(dom, 0) + FLOPS_PER_TRI * tris.get(dom, 0)
            per_launch_flops = flops / launches[dom]
            achieved = per_launch_flops / (dom_avg_ms * 1e-3) / 1e12
            roofline = {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "flops_per_launch": per_launch_flops,
                        # wave64 VALU instructions issued per CU cycle (1.0 = the non-packed issue limit)
                        "valu_issue_per_cu_cycle": measured_traffic(kname, "valu_per_cu_cycle"),
                        "l2_hit_rate": measured_traffic(kname, "l2_hit_rate"),
                        "node_visits_per_frame": nodes.get(dom, 0) / args.steps,
                        "tri_tests_per_frame": tris.get(dom, 0) / args.steps, **common}
        else:
            roofline = {"bound": "hbm", "achieved": state_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": state_gbs / HBM_PEAK_GBS, "bytes_per_launch": per_launch_bytes, **common}
        state_bytes = sum(nbytes.values()) / args.steps
        state_floor = {"bytes_per_frame": state_bytes,
                       "frac_of_frame": (state_bytes / (res["wave"]["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS)
                       if "wave" in res else None}

    head = "wave" if "wave" in inflight else "mega"
    out = {
        "metric": "path samples/s wavefront vs megakernel @1080p, 1M tris; adjoint samples/s",
        "value": inflight[head]["value"],
        "unit": "path-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": inflight[head]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"procedural scene {nt} triangles (1000 icospheres + 1000 tessellated boxes, "
                               f"ground, 16 quad lights), {W}x{H}, {SPP} spp/frame, max depth {DEPTH}, "
                               f"roulette from {RR}, light sampling on; {head} schedule, progressive frames with "
                               f"three in flight (bit-identical to frame by frame)",
                   "width": W, "height": H, "spp": SPP, "max_depth": DEPTH, "triangles": nt},
        "schedules": {m: {"frames_in_flight": inflight[m], "frame_by_frame": {"value": res[m]["value"],
                                                                                 "ms_per_step": res[m]["ms"]}}
                      for m in modes},
        "wave_over_mega": ({"frames_in_flight": inflight["wave"]["value"] / inflight["mega"]["value"],
                            "frame_by_frame": res["wave"]["value"] / res["mega"]["value"]} if len(res) == 2 else None),
        "rays_per_s": ((ext_rays_per_frame + sh_rays_per_frame) / (inflight["wave"]["ms_per_step"] * 1e-3))
                      if "wave" in inflight else None,
        "rays_per_frame": {"extension": ext_rays_per_frame, "shadow": sh_rays_per_frame},
        "stage_ms_per_frame": frame_stage_ms,
        "launch_params": {"frame_by_frame": tuned, "frames_in_flight": tuned_inflight},
        "roofline": roofline,
        "state_traffic": state_floor,
        "stage_items_per_frame": {k: v / args.steps for k, v in items.items()},
        "node_visits_per_frame": {k: v / args.steps for k, v in nodes.items()},
        "tri_tests_per_frame": {k: v / args.steps for k, v in tris.items()},
        "paper_context": "paper reports ~16% (1.138x by its table) wavefront over megakernel on an RTX 3060 Ti "
                         "with RT cores, A Beautiful Game scene",
    }

    out["hbm_copy_ceiling"] = copy_ceiling(torch)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_bench(ptmi, scenes, scene, torch, args)

    if not args.no_cpu:
        log("oracle CPU baseline ...")
        out["cpu_baseline"] = cpu_baseline(scene, cam)
    print(json.dumps(out), flush=True)


def batch_bench(args):
    """64 jobs: per job a procedural scene of T triangles (T log-uniform in
    [1e4, 2e6]), a resolution from {256^2, 512^2, 1024^2, 1920x1080}, 1..8
    spp, depth 8, roulette from 3; all in one batched persistent wavefront."""
    import numpy as np
    import torch

    from paper_2605_27323_amd import autotune, ptmi, scenes
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
    opts = {} if args.no_tune else autotune.tune_batch(Rs, job_args, cache=None, log=log)
    log(f"batch options {opts}")
    ws = None
    _, _, r = ptmi.render_batch(Rs, job_args, **opts)
    ws = r["workspace"]
    runs = []
    for _ in range(max(1, args.steps // 16)):
        _, ms, r = ptmi.render_batch(Rs, job_args, workspace=ws, **opts)
        runs.append((r["seconds"], ms))
    sec = min(t for t, _ in runs)
    ms = [m for t, m in runs if t == sec][0]
    out = {"metric": "batched path samples/s (64 jobs)", "value": total / sec, "unit": "path-samples/s",
           "n_gpus": 1, "steps": len(runs), "warmup": 1, "ms_per_step": sec * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"64 jobs, {ntri} triangles in total, {total} path samples, depth {DEPTH}, "
                                  f"roulette from {RR}, one batched persistent wavefront with a hipGraph loop",
                      "triangles": ntri, "path_samples": total},
           "job_latency_ms": {"p50": float(np.percentile(ms, 50)), "p99": float(np.percentile(ms, 99)),
                              "max": float(np.max(ms))},
           "iterations": r["iterations"], "graph_launches": r["launches"], "batch_options": opts}
    print(json.dumps(out), flush=True)


def divergence_bench(args):
    """~10M triangles, 64 material ids (Lambertian, conductor, rough
    dielectric, emissive), 1920x1080, 4 spp, depth 16, roulette from 3:
    megakernel, wavefront, wavefront with the material sort, the ray sort,
    and the wavefront and megakernel with three frames in flight."""
    import torch

    from paper_2605_27323_amd import ptmi, scenes
    t0 = time.perf_counter()
    scene, cam = scenes.procedural(seed=3, n_objects=20000, width=W, height=H, material_mode="divergence")
    nt = scene["indices"].shape[0]
    R = ptmi.Renderer(scene, cam, max_leaf=args.max_leaf)
    log(f"divergence scene {nt} triangles, BVH depth {R.info.depth} (setup {time.perf_counter() - t0:.1f} s)")
    kw = dict(spp=4, max_depth=16, rr_start=3, nee=True, seed=0)
    img = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    res = {}
    k = max(2, args.steps // 8)
    given = json.loads(args.params) if args.params else {}
    wave = dict(given.get("wave", DIVERGENCE_PARAMS["wave"]))
    mega = dict(given.get("mega", DIVERGENCE_PARAMS["mega"]))
    def sorted_by(flag):
        return dict(wave, mode="wave", flags=wave.get("flags", 0) | flag,
                    sort_threshold=wave.get("sort_threshold", 1 << 16))

    runs = [("mega", dict(mode="mega", **mega)), ("wave", dict(mode="wave", **wave)),
            ("wave_material_sort", sorted_by(ptmi.FLAG_SORT_MATERIAL)),
            ("wave_ray_sort", sorted_by(ptmi.FLAG_SORT_RAYS))]
    for name, extra in runs:
        R.render(out=img, frame=0, **kw, **extra)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(k):
            R.render(out=img, frame=1 + i, **kw, **extra)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / k
        res[name] = {"ms_per_frame": dt * 1e3, "path_samples_per_s": W * H * 4 / dt}
        log(f"{name}: {dt * 1e3:.2f} ms/frame")
    for name, extra in [("mega_in_flight", dict(mode="mega", **mega)), ("wave_in_flight", dict(mode="wave", **wave))]:
        R.render_frames(2, out=img, frame=0, **kw, **extra)
        torch.cuda.synchronize()
        t = time.perf_counter()
        R.render_frames(k, out=img, frame=2, **kw, **extra)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / k
        res[name] = {"ms_per_frame": dt * 1e3, "path_samples_per_s": W * H * 4 / dt}
        log(f"{name}: {dt * 1e3:.2f} ms/frame")
    best = max((r for r in res if r.startswith("wave")), key=lambda r: res[r]["path_samples_per_s"])
    out = {"metric": "path samples/s, divergence workload", "value": res[best]["path_samples_per_s"],
           "unit": "path-samples/s", "n_gpus": 1, "steps": k, "warmup": 1,
           "ms_per_step": res[best]["ms_per_frame"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"procedural {nt} triangles, 64 material ids, {W}x{H}, 4 spp, depth 16, "
                                  f"roulette from 3; best wavefront schedule: {best}"}, "schedules": res}
    print(json.dumps(out), flush=True)


def adjoint_bench(ptmi, scenes, scene, torch, args):
    """Backward (path replay) of the 512x512, 8 spp, depth 6 frame."""
    cam = dict(eye=(0.0, 50.0, -130.0), target=(0.0, 40.0, 0.0), up=(0.0, 1.0, 0.0), vfov_deg=50.0,
               width=512, height=512)
    try:
        R = ptmi.Renderer(scene, cam, max_leaf=args.max_leaf)
        kw = dict(spp=8, max_depth=6, rr_start=-1, nee=True, seed=0)
        d_img = torch.ones((512, 512, 3), dtype=torch.float32, device="cuda")
        ga = torch.zeros_like(R.albedo)
        ge = torch.zeros_like(R.emission)
        R.backward(d_img, ga, ge, **kw)
        torch.cuda.synchronize()
        k = max(4, args.steps // 8)
        t = time.perf_counter()
        for i in range(k):
            R.backward(d_img, ga, ge, frame=i, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        n = 512 * 512 * 8 * k
        log(f"adjoint: {dt * 1e3 / k:.3f} ms per backward, {n / dt / 1e6:.1f} M samples/s")
        return {"value": n / dt, "unit": "adjoint samples/s", "ms_per_backward": dt * 1e3 / k,
                "config": "same scene, 512x512, 8 spp, max depth 6, roulette off"}
    except ptmi.PtError as e:
        log(f"adjoint unavailable: {e}")
        return None


if __name__ == "__main__":
    main()
