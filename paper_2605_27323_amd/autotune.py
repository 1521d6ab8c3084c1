"""Autotuner for the render launch parameters.

Successive halving: every candidate is timed on a short proxy run, the
faster half is kept and re-timed with twice the repetitions, until one is
left.  Results are cached in a JSON file keyed by the device, the workload
shape and the schedule, so a later run with the same key reuses them.  Any
parameter point renders the same image bit for bit (the parity tests check
it), so tuning changes speed only.
"""
from __future__ import annotations

import itertools
import json
import os
import time

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ptmi_autotune.json")

FRAME_SPACE = {
    "wave": {"block": [64, 128, 256], "grid_mult": [4, 8, 16], "stack_lds": [8, 16, 24, 32],
             "sort_threshold": [None, 1 << 16], "ray_sort": [False, True],
             "tail_threshold": [0, 1 << 16, 1 << 18, 1 << 19, 1 << 20]},
    "mega": {"block": [64, 128, 256], "grid_mult": [2, 4, 8, 16], "stack_lds": [8, 16, 24, 32],
             "mega_waves": [4, 5]},
}
# tried after the other wave parameters are chosen (0 = off)
TAIL_BOUNCES = [0, 2, 3, 4, 5, 6]
# The batched launch has no sort or hybrid-tail stage, so its space is the
# pool (capacity, count) and the launch shape.
BATCH_SPACE = {"pool_capacity": [1 << 20, 1 << 21, 1 << 22, 1 << 23, 1 << 24], "block": [128, 256],
               "grid_mult": [4, 8, 16], "stack_lds": [8, 16, 32], "pools": [1, 2, 3, 4]}


def _bucket(x):
    return int(2 ** round(__import__("math").log2(max(1, x))))


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, key, value):
    d = _load(path)
    d[key] = value
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def successive_halving(candidates, measure, reps0=1, log=None):
    """candidates: list of dicts; measure(cand, reps) -> seconds per rep."""
    pool = list(candidates)
    reps = reps0
    history = []
    while len(pool) > 1:
        timed = sorted(((measure(c, reps), i, c) for i, c in enumerate(pool)), key=lambda t: (t[0], t[1]))
        history.append([(t, c) for t, _, c in timed])
        if log:
            log(f"round reps={reps}: best {timed[0][0] * 1e3:.3f} ms {timed[0][2]}, kept {max(1, len(pool) // 2)}")
        pool = [c for _, _, c in timed[:max(1, len(pool) // 2)]]
        reps *= 2
    return pool[0], history


def _device_name(torch):
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"


def tune_frame(renderer, mode="wave", cache=DEFAULT_CACHE, space=None, log=None, in_flight=False, **kw):
    """Best launch parameters for renderer.render(mode=mode, **kw), or with
    in_flight for renderer.render_frames (frames in flight)."""
    import torch

    from . import ptmi
    key = json.dumps(["frame", _device_name(torch), mode, _bucket(renderer.nt), renderer.width, renderer.height,
                      kw.get("spp", 1), kw.get("max_depth", 5), kw.get("rr_start", -1), bool(in_flight)])
    hit = _load(cache).get(key) if cache else None
    if hit:
        return hit
    space = space or FRAME_SPACE[mode]
    names = list(space)
    cands = []
    for vals in itertools.product(*(space[n] for n in names)):
        c = dict(zip(names, vals))
        flags = 0
        if c.pop("ray_sort", False):
            flags |= ptmi.FLAG_SORT_RAYS
        if c.get("sort_threshold", None) is None:
            c.pop("sort_threshold", None)
        else:
            flags |= ptmi.FLAG_SORT_MATERIAL
        if flags & ptmi.FLAG_SORT_RAYS and "sort_threshold" not in c:
            c["sort_threshold"] = 1 << 16
        if flags:
            c["flags"] = flags
        cands.append(c)
    img = torch.empty((renderer.height, renderer.width, 3), dtype=torch.float32, device=renderer.torch_device)

    rest = {k: v for k, v in kw.items() if k != "frame"}

    def measure(c, reps):
        if in_flight:
            n = max(6, 2 * reps)  # long enough for the pipeline to fill
            renderer.render_frames(2, out=img, mode=mode, frame=0, **rest, **c)
            torch.cuda.synchronize()
            t = time.perf_counter()
            renderer.render_frames(n, out=img, mode=mode, frame=2, **rest, **c)
            torch.cuda.synchronize()
            return (time.perf_counter() - t) / n
        renderer.render(out=img, mode=mode, **kw, **c)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(reps):
            renderer.render(out=img, mode=mode, frame=1 + i, **rest, **c)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    best, _ = successive_halving(cands, measure, log=log)
    if mode == "wave" and space is FRAME_SPACE[mode]:
        # then the bounce from which the hybrid tail finishes every path;
        # the candidates differ by a few per cent, so each is timed over
        # as many frames as the last rounds of the first stage
        depth = kw.get("max_depth", 5)
        tbs = [t for t in TAIL_BOUNCES if t <= depth]
        best, _ = successive_halving([dict(best, tail_bounce=t) for t in tbs], measure, reps0=32, log=log)
        if best.get("tail_threshold", 0) or best.get("tail_bounce", 0):
            # and whether the tail spreads its queue over partly filled waves
            best, _ = successive_halving([dict(best, tail_spread=v) for v in (False, True)], measure, reps0=32,
                                         log=log)
    if cache:
        _store(cache, key, best)
    return best


def tune_batch(renderers, job_args, cache=DEFAULT_CACHE, space=None, log=None):
    """Best batch options for ptmi.render_batch(renderers, job_args, ...)."""
    import torch

    from . import ptmi
    total = sum(R.width * R.height * a.get("spp", 1) for R, a in zip(renderers, job_args))
    key = json.dumps(["batch", _device_name(torch), len(renderers), _bucket(total),
                      _bucket(sum(R.nt for R in renderers))])
    hit = _load(cache).get(key) if cache else None
    if hit:
        return hit
    space = space or BATCH_SPACE
    names = list(space)
    cands = [dict(zip(names, vals)) for vals in itertools.product(*(space[n] for n in names))]
    # every pool needs a job and 64 slots
    cands = [c for c in cands if c.get("pools", 1) <= len(renderers)
             and c.get("pool_capacity", 1 << 21) // max(1, c.get("pools", 1)) >= 64]
    # proxy: the same jobs at 1 spp
    proxy = [dict(a, spp=1) for a in job_args]
    ws = [None]

    def measure(c, reps):
        t = 0.0
        for _ in range(reps):
            _, _, res = ptmi.render_batch(renderers, proxy, workspace=ws[0], **c)
            ws[0] = res["workspace"]
            t += res["seconds"]
        return t / reps

    best, _ = successive_halving(cands, measure, log=log)
    if cache:
        _store(cache, key, best)
    return best
