"""Vertex attributes and the coated material on the GPU (paper Sec. 2.3: the
shading stage interpolates the hit's vertex normals and texture coordinates;
Sec. 3: a layered material, here a coat over a Lambertian base): megakernel,
wavefront and hybrid-tail images against the oracle, full images of small
scenes and sampled pixels of the 1.02M-triangle procedural scene with
attributes in the benchmark's launch configurations; the adjoint and the
batched launch with attribute scenes against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2605_27323_amd import scenes
from tests._parity import assert_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2605_27323_amd import ptmi  # noqa: E402


def log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("cfg", [dict(spp=4, max_depth=6, rr_start=3, seed=5, frame=1),
                                 dict(spp=2, max_depth=4, nee=False, seed=2)])
def test_cornell_attributes_all_pixels(cfg):
    scene, cam = scenes.cornell_attributes(coat=(0.3, 1.5))
    cam = dict(cam, width=96, height=80)
    log("cornell attributes", cfg)
    R = ptmi.Renderer(scene, cam)
    assert R.info.attribute_bytes == 64 * scene["indices"].shape[0]
    mega = R.render(mode="mega", **cfg).cpu().numpy()
    wave = R.render(mode="wave", **cfg).cpu().numpy()
    hybrid = R.render(mode="wave", tail_bounce=2, tail_threshold=2000, **cfg).cpu().numpy()
    sort = R.render(mode="wave", flags=ptmi.FLAG_SORT_MATERIAL, sort_threshold=1, **cfg).cpu().numpy()
    torch.cuda.synchronize()
    for img in (wave, hybrid, sort):
        assert np.array_equal(mega.view(np.uint32), img.view(np.uint32))
    o, frag = oracle.Scene(scene).render(cam, **cfg)
    nexact = assert_parity(wave.reshape(-1, 3), o, frag, what=f"cornell attributes {cfg}")
    assert nexact >= 0.999 * o.shape[0]


def test_instanced_attributes_all_pixels():
    sc, inst, cam = scenes.instanced_procedural(seed=9, n_instances=120, n_meshes=10, width=64, height=40,
                                                attributes=True)
    cfg = dict(spp=2, max_depth=6, rr_start=3, seed=5, frame=1)
    log("instanced attributes", cfg)
    R = ptmi.Renderer(sc, cam, instances=inst)
    mega = R.render(mode="mega", **cfg).cpu().numpy()
    wave = R.render(mode="wave", tail_bounce=2, tail_threshold=300, **cfg).cpu().numpy()
    assert np.array_equal(mega.view(np.uint32), wave.view(np.uint32))
    o, frag = oracle.Scene(sc, instances=inst).render(cam, **cfg)
    nexact = assert_parity(wave.reshape(-1, 3), o, frag, what="instanced attributes")
    assert nexact >= 0.999 * o.shape[0]


def test_procedural_attributes_full_size_sampled_pixels():
    # the 1.02M-triangle scene with smooth-shaded icospheres, checker
    # textures and coats at 1920x1080, in the benchmark's launch
    # configurations, against the oracle on sampled pixels
    scene, cam = scenes.procedural(seed=2, n_objects=2000, attributes=True)
    R = ptmi.Renderer(scene, cam)
    log("procedural attributes full size", R.nt, "triangles")
    px = scenes.pixel_subset(1920, 1080, 2048, seed=78)
    cfg = dict(spp=1, max_depth=8, rr_start=3, nee=True, seed=0, frame=2)
    wave = R.render(mode="wave", block=256, grid_mult=8, stack_lds=8, tail_threshold=1 << 19, tail_bounce=3,
                    **cfg).cpu().numpy()
    mega = R.render(mode="mega", block=256, grid_mult=8, stack_lds=8, mega_waves=5, **cfg).cpu().numpy()
    pure = R.render(mode="wave", block=128, grid_mult=8, stack_lds=8, **cfg).cpu().numpy()
    assert np.array_equal(mega.view(np.uint32), wave.view(np.uint32))
    assert np.array_equal(pure.view(np.uint32), wave.view(np.uint32))
    o, frag = oracle.Scene(scene).render(cam, pixels=px, **cfg)
    assert_parity(wave.reshape(-1, 3)[px], o, frag, what="procedural attributes 1M")


def test_adjoint_with_attributes_matches_oracle():
    scene, cam = scenes.cornell_attributes(coat=(0.3, 1.5))
    cam = dict(cam, width=48, height=40)
    R = ptmi.Renderer(scene, cam)
    rng = np.random.default_rng(2)
    d = rng.normal(size=(40 * 48, 3)).astype(np.float32)
    ga = torch.zeros_like(R.albedo)
    ge = torch.zeros_like(R.emission)
    kw = dict(spp=2, max_depth=4, seed=3)
    R.backward(torch.from_numpy(d).cuda(), ga, ge, **kw)
    torch.cuda.synchronize()
    oa, oe, aa, ae = oracle.Scene(scene).backward(cam, d, **kw)
    for g, o, a in [(ga.cpu().numpy()[:R.nt].astype(np.float64), oa, aa),
                    (ge.cpu().numpy()[:R.nt].astype(np.float64), oe, ae)]:
        # atomics sum in any order: 1e-4 of the summed absolute terms
        assert (np.abs(g - o) <= 1e-4 * a + 1e-7 * np.abs(o).max()).all()
        assert np.linalg.norm(g - o) <= 1e-4 * np.linalg.norm(o)
    assert np.abs(oa[scene["tri_mat"] == 1]).sum() > 0


def test_batch_with_attribute_job_matches_oracle():
    s0, c0 = scenes.cornell_attributes(coat=(0.2, 1.4))
    c0 = dict(c0, width=40, height=32)
    s1, c1 = scenes.procedural(seed=1001, n_objects=30, width=48, height=32, attributes=True)
    s2, c2 = scenes.procedural(seed=1002, n_objects=30, width=32, height=24)
    rs = [ptmi.Renderer(s, c) for s, c in ((s0, c0), (s1, c1), (s2, c2))]
    args = [dict(spp=2, max_depth=5, rr_start=3, seed=5, frame=1), dict(spp=1, max_depth=6, rr_start=3, seed=6),
            dict(spp=2, max_depth=4, seed=7)]
    imgs, _, _ = ptmi.render_batch(rs, args, pool_capacity=4096)
    torch.cuda.synchronize()
    for j, ((s, c), kw) in enumerate(zip(((s0, c0), (s1, c1), (s2, c2)), args)):
        o, frag = oracle.Scene(s).render(c, job=j, **kw)
        assert_parity(imgs[j].cpu().numpy().reshape(-1, 3), o, frag, what=f"attribute batch job {j}")


def test_coat_without_attributes_matches_oracle():
    # coated materials alone select the extended shading kernels
    scene, cam = scenes.cornell()
    scene = {k: v.copy() for k, v in scene.items()}
    scene["materials"] = np.array([[0, 1.0, 1.5, 0], [scenes.COATED, 0.2, 1.6, 0]], np.float32)
    scene["tri_mat"][10:22] = 1
    cam = dict(cam, width=64, height=48)
    cfg = dict(spp=4, max_depth=6, rr_start=3, seed=4)
    R = ptmi.Renderer(scene, cam)
    mega = R.render(mode="mega", **cfg).cpu().numpy()
    wave = R.render(mode="wave", tail_bounce=2, tail_threshold=500, **cfg).cpu().numpy()
    assert np.array_equal(mega.view(np.uint32), wave.view(np.uint32))
    o, frag = oracle.Scene(scene).render(cam, **cfg)
    nexact = assert_parity(wave.reshape(-1, 3), o, frag, what="coat without attributes")
    assert nexact >= 0.999 * o.shape[0]
