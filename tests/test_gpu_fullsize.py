"""Parity at the workloads' full sizes, in the launch configurations the
benchmark times, on outputs the oracle computes one by one:

* divergence workload (~10M triangles, 64 material ids with rough
  dielectrics and emitters, 1920x1080, 4 spp, depth 16, roulette from 3):
  sampled pixels of the megakernel and the wavefront (frame by frame, with
  the material and ray sorts, frames in flight) against the oracle;
* adjoint workload (the 1M-triangle scene at 512x512, 8 spp, depth 6):
  the gradient of an image loss that weights sampled pixels only, against
  the oracle's binary64 adjoint over those pixels;
* batched workload (64 jobs, ~30M triangles): sampled jobs of one batched
  launch equal, bit for bit, the same jobs rendered alone (whose parity with
  the oracle the other tests establish).

Bars as in the other parity tests.
"""
import numpy as np
import pytest

import oracle
from paper_2605_27323_amd import scenes
from tests._parity import assert_parity, oracle_image

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2605_27323_amd import ptmi  # noqa: E402

W, H = 1920, 1080
# the benchmark's launch parameters (bench.py FIXED_PARAMS / DIVERGENCE_PARAMS)
DIV_WAVE = dict(block=256, grid_mult=8, stack_lds=8, tail_threshold=1 << 18, tail_bounce=6)
DIV_MEGA = dict(block=256, grid_mult=4, stack_lds=8)
WAVE = dict(block=256, grid_mult=8, stack_lds=8, tail_threshold=1 << 18, tail_bounce=4)


def log(*a):
    print(*a, flush=True)


def test_divergence_full_size_sampled_pixels():
    scene, cam = scenes.procedural(seed=3, n_objects=20000, width=W, height=H, material_mode="divergence")
    log("divergence", scene["indices"].shape[0], "tris 1920x1080 spp 4 depth 16")
    R = ptmi.Renderer(scene, cam)
    cfg = dict(spp=4, max_depth=16, rr_start=3, nee=True, seed=0, frame=2)
    wave = R.render(mode="wave", **cfg, **DIV_WAVE).cpu().numpy()
    mega = R.render(mode="mega", **cfg, **DIV_MEGA).cpu().numpy()
    assert np.array_equal(mega.view(np.uint32), wave.view(np.uint32))
    for flags in (ptmi.FLAG_SORT_MATERIAL, ptmi.FLAG_SORT_RAYS):
        srt = R.render(mode="wave", flags=flags, **cfg, **DIV_WAVE).cpu().numpy()
        assert np.array_equal(srt.view(np.uint32), wave.view(np.uint32)), flags
    kw = {k: v for k, v in cfg.items() if k != "frame"}
    inflight = R.render_frames(3, mode="wave", frame=0, **kw, **DIV_WAVE).cpu().numpy()
    assert np.array_equal(inflight.view(np.uint32), wave.view(np.uint32))
    torch.cuda.synchronize()
    log("oracle BVH over", scene["indices"].shape[0], "triangles")
    S = oracle.Scene(scene)
    px = scenes.pixel_subset(W, H, 2048, seed=77)
    ref, frag = S.render(cam, pixels=px, **cfg)
    assert_parity(wave.reshape(-1, 3)[px], ref, frag, what="divergence 10M")


def test_adjoint_full_size_sampled_pixels():
    scene, _ = scenes.procedural(seed=2, n_objects=2000)
    cam = dict(eye=(0.0, 50.0, -130.0), target=(0.0, 40.0, 0.0), up=(0.0, 1.0, 0.0), vfov_deg=50.0,
               width=512, height=512)
    log("adjoint 1M 512x512 spp 8 depth 6")
    R = ptmi.Renderer(scene, cam)
    px = scenes.pixel_subset(512, 512, 256, seed=5)
    d = np.random.default_rng(6).normal(size=(px.size, 3)).astype(np.float32)
    d_full = np.zeros((512 * 512, 3), np.float32)
    d_full[px] = d
    kw = dict(spp=8, max_depth=6, rr_start=-1, nee=True, seed=0, frame=1)
    ga = torch.zeros_like(R.albedo)
    ge = torch.zeros_like(R.emission)
    R.backward(torch.from_numpy(d_full).cuda(), ga, ge, **kw)
    ga, ge = ga.cpu().numpy()[:R.nt], ge.cpu().numpy()[:R.nt]
    oa, oe, aa, ae = oracle.Scene(scene).backward(cam, d, pixels=px, **{k: v for k, v in kw.items()
                                                                          if k != "rr_start"})
    touched = 0
    for g, o, a in [(ga, oa, aa), (ge, oe, ae)]:
        err = np.abs(g.astype(np.float64) - o)
        bound = 1e-4 * a + 1e-7 * np.abs(o).max()
        assert (err <= bound).all(), (err.max(), int((err > bound).sum()))
        assert np.linalg.norm(g - o) <= 1e-4 * np.linalg.norm(o)
        touched += int((o != 0).any(1).sum())
    log("triangles with a gradient:", touched)
    assert touched > 100


def test_batch_full_size_sampled_jobs():
    specs = scenes.batch_jobs(seed=4, n_jobs=64)
    Rs, args, sc_all = [], [], []
    for j, sp in enumerate(specs):
        sc, cam = scenes.procedural(seed=sp["scene_seed"], n_objects=sp["n_objects"], width=sp["width"],
                                    height=sp["height"])
        Rs.append(ptmi.Renderer(sc, cam))
        args.append(dict(spp=sp["spp"], max_depth=8, rr_start=3, nee=True, seed=0, job=j))
        sc_all.append((sc, cam) if j in (7, 31, 63) else None)
    log("batch 64 jobs", sum(R.nt for R in Rs), "triangles")
    imgs, ms, res = ptmi.render_batch(Rs, args, pool_capacity=1 << 22, block=256, grid_mult=8, stack_lds=8)
    torch.cuda.synchronize()
    assert res["path_samples"] == sum(R.width * R.height * a["spp"] for R, a in zip(Rs, args))
    # the largest, the smallest and a few other jobs
    sizes = [R.nt for R in Rs]
    pick = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 7, 31, 63})
    for j in pick:
        ref = Rs[j].render(mode="wave", **args[j], **WAVE).cpu().numpy()
        assert np.array_equal(imgs[j].cpu().numpy().view(np.uint32), ref.view(np.uint32)), j
    log("jobs compared:", pick)
    # against the oracle: 1024 sampled pixels of jobs 7, 31 and 63 (job != 0
    # keys their random numbers)
    for j in (7, 31, 63):
        sc, cam = sc_all[j]
        px = scenes.pixel_subset(cam["width"], cam["height"], 1024, seed=1234 + j)
        ref, frag, _ = oracle_image(sc, cam, pixels=px, **args[j])
        got = imgs[j].cpu().numpy().reshape(-1, 3)[px]
        assert_parity(got, ref, frag, what=f"batch job {j} ({Rs[j].nt} triangles) vs oracle")
