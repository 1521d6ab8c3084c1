"""Two-level scenes on the GPU (paper Sec. 2.3 and 3: a top-level structure
over instances of per-mesh structures): megakernel and wavefront images of
instanced scenes against the oracle's instanced path loop; a flat scene cut
into identity instances renders the flat image bit for bit; the adjoint and
the batched launch reject instanced scenes."""
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


@pytest.mark.parametrize("cfg", [dict(spp=2, max_depth=6, rr_start=3, seed=5, frame=1),
                                 dict(spp=1, max_depth=3, nee=False, seed=2)])
def test_instanced_small_all_pixels(cfg):
    sc, inst, cam = scenes.instanced_procedural(seed=9, n_instances=120, n_meshes=10, width=64, height=40)
    log("instanced small", cfg)
    R = ptmi.Renderer(sc, cam, instances=inst)
    assert R.info.instance_count == len(inst["inst_mesh"])
    mega = R.render(mode="mega", **cfg).cpu().numpy()
    wave = R.render(mode="wave", **cfg).cpu().numpy()
    hybrid = R.render(mode="wave", tail_bounce=2, tail_threshold=300, **cfg).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(mega.view(np.uint32), wave.view(np.uint32))
    assert np.array_equal(hybrid.view(np.uint32), wave.view(np.uint32))
    o, frag = oracle.Scene(sc, instances=inst).render(cam, **cfg)
    nexact = assert_parity(wave.reshape(-1, 3), o, frag, what=f"instanced {cfg}")
    assert nexact >= 0.999 * o.shape[0]


def test_identity_instances_equal_flat_scene():
    sc, cam = scenes.procedural(seed=21, n_objects=40, width=48, height=32)
    cfg = dict(spp=2, max_depth=6, rr_start=3, seed=5, frame=1)
    flat = ptmi.Renderer(sc, cam).render(mode="wave", **cfg).cpu().numpy()
    for parts in (1, 6):
        R = ptmi.Renderer(sc, cam, instances=scenes.split_into_instances(sc, parts))
        for mode in ("mega", "wave"):
            img = R.render(mode=mode, **cfg).cpu().numpy()
            assert np.array_equal(img.view(np.uint32), flat.view(np.uint32)), (parts, mode)


def test_instanced_full_size_sampled_pixels():
    # ~1M instanced triangles (4016 instances of 34 meshes) at 1920x1080, the
    # benchmark's launch configurations, against the oracle on sampled pixels
    sc, inst, cam = scenes.instanced_procedural()
    R = ptmi.Renderer(sc, cam, instances=inst)
    log("instanced full size", R.info.instance_count, "instances", R.nt, "unique triangles")
    px = scenes.pixel_subset(1920, 1080, 2048, seed=77)
    cfg = dict(spp=1, max_depth=8, rr_start=3, nee=True, seed=0, frame=3)
    wave = R.render(mode="wave", block=256, grid_mult=4, stack_lds=8, tail_threshold=1 << 18, tail_bounce=3,
                    **cfg).cpu().numpy()
    mega = R.render(mode="mega", block=256, grid_mult=4, stack_lds=8, mega_waves=5, **cfg).cpu().numpy()
    pure = R.render(mode="wave", **cfg).cpu().numpy()
    assert np.array_equal(mega.view(np.uint32), wave.view(np.uint32))
    assert np.array_equal(pure.view(np.uint32), wave.view(np.uint32))
    o, frag = oracle.Scene(sc, instances=inst).render(cam, pixels=px, **cfg)
    assert_parity(wave.reshape(-1, 3)[px], o, frag, what="instanced 1M")


def test_instanced_scene_rejected_by_adjoint_and_batch():
    sc, inst, cam = scenes.instanced_procedural(seed=9, n_instances=20, n_meshes=4, width=16, height=16)
    R = ptmi.Renderer(sc, cam, instances=inst)
    ga = torch.zeros_like(R.albedo)
    ge = torch.zeros_like(R.emission)
    with pytest.raises(ptmi.PtError) as e:
        R.backward(torch.ones((16, 16, 3), device="cuda"), ga, ge, spp=1, max_depth=2)
    assert e.value.code == ptmi.PT_EUNSUPPORTED
    with pytest.raises(ptmi.PtError) as e:
        ptmi.render_batch([R], [dict(spp=1, max_depth=2)])
    assert e.value.code == ptmi.PT_EUNSUPPORTED
