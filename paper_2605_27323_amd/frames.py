"""Render frames of the 1.02M-triangle procedural scene (1920x1080, 1 spp,
depth 8, roulette from bounce 3) with given launch parameters and print one
JSON line with the rays and traversal work they took: a fixed workload for
profiler runs, whose per-dispatch counters are divided by these totals
(for example HBM bytes or VALU instructions per extension ray).

    python3 frames.py [--root CHECKOUT] [--mode wave|mega] [--params JSON]
                      [--frames K] [--work-frames J]

--root renders with the package of another checkout of this project (same
Python interface: an older revision, to compare kernels before and after a
change on the same workload).  The first K frames run without work counters
(the kernels a profiler should attribute); then J frames with
FLAG_COUNT_WORK (kernels compiled with counters, other names) give node
visits and triangle tests per ray.
"""
import argparse
import json
import os
import sys
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--root", default=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap.add_argument("--mode", default="wave", choices=["wave", "mega"])
    ap.add_argument("--params", default="{}", help="launch parameters as JSON, e.g. {\"grid_mult\": 8}")
    ap.add_argument("--frames", type=int, default=4)
    ap.add_argument("--work-frames", type=int, default=2)
    args = ap.parse_args()
    sys.path.insert(0, os.path.abspath(args.root))
    import torch
    from paper_2605_27323_amd import ptmi, scenes

    scene, cam = scenes.procedural(seed=2, n_objects=2000, width=1920, height=1080)
    R = ptmi.Renderer(scene, cam)
    p = json.loads(args.params)
    kw = dict(spp=1, max_depth=8, rr_start=3, nee=True, seed=0, mode=args.mode, **p)
    img = torch.empty((1080, 1920, 3), dtype=torch.float32, device="cuda")
    out = {"root": os.path.abspath(args.root), "mode": args.mode, "params": p, "frames": args.frames,
           "triangles": int(scene["indices"].shape[0]), "extension_rays": 0, "shadow_rays": 0}
    t = time.perf_counter()
    for f in range(args.frames):
        R.render(out=img, frame=f, **kw)
        st = R.stats()
        out["extension_rays"] += st["extension_rays"]
        out["shadow_rays"] += st["shadow_rays"]
    torch.cuda.synchronize()
    out["ms_per_frame_with_stats"] = (time.perf_counter() - t) * 1e3 / max(1, args.frames)
    nodes, tris, rays = {}, {}, [0, 0]
    for f in range(args.work_frames):
        R.render(out=img, frame=f, flags=ptmi.FLAG_COUNT_WORK, **kw)
        st = R.stats()
        rays[0] += st["extension_rays"]
        rays[1] += st["shadow_rays"]
        for k, v in st["node_visits"].items():
            nodes[k] = nodes.get(k, 0) + v
        for k, v in st["tri_tests"].items():
            tris[k] = tris.get(k, 0) + v
    out["work_frames"] = {"frames": args.work_frames, "extension_rays": rays[0], "shadow_rays": rays[1],
                          "node_visits": nodes, "tri_tests": tris}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
