"""The allocation-free entry point (pt_render_frame_noalloc, the library's
own per-GPU scratch instead of a caller workspace) against pt_render_frame:
two calls in a row, the second with a smaller input, bit for bit; and the
megakernel image against the oracle."""
import numpy as np
import pytest

from paper_2605_27323_amd import scenes
from tests._parity import assert_parity, oracle_image

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2605_27323_amd import ptmi  # noqa: E402


def log(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("seed,n_objects", [(5, 150), (6, 8)])
def test_noalloc_equals_render_frame(seed, n_objects):
    # a deep BVH (spill area in use with stack_lds 8) and a shallow one
    scene, cam = scenes.procedural(seed=seed, n_objects=n_objects, width=96, height=64)
    R = ptmi.Renderer(scene, cam)
    log("noalloc", seed, n_objects, "stack entries", R.info.stack_entries)
    kw = dict(max_depth=6, rr_start=3, seed=9, block=256, grid_mult=2, stack_lds=8)
    for (w, h, spp, frame) in [(96, 64, 3, 0), (40, 24, 2, 5)]:  # the second call is smaller
        c = dict(cam, width=w, height=h)
        R.set_camera(c)
        acc_a = torch.full((h, w, 3), 0.25, device="cuda")
        acc_b = acc_a.clone()
        ref = R.render(mode="mega", spp=spp, frame=frame, accum=acc_a, **kw)
        got = R.render_noalloc(spp=spp, frame=frame, accum=acc_b, **kw)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy().view(np.uint32), ref.cpu().numpy().view(np.uint32)), (w, h)
        assert np.array_equal(acc_b.cpu().numpy().view(np.uint32), acc_a.cpu().numpy().view(np.uint32)), (w, h)
        st = R.stats()
        assert st["extension_rays"] > 0
        o, frag, _ = oracle_image(scene, c, spp=spp, frame=frame, max_depth=6, rr_start=3, seed=9)
        assert_parity(got.cpu().numpy(), o, frag, what=f"noalloc {w}x{h}")


def test_noalloc_rejections():
    scene, cam = scenes.procedural(seed=5, n_objects=150, width=64, height=48)
    R = ptmi.Renderer(scene, cam)
    with pytest.raises(ptmi.PtError) as e:
        R.render_noalloc(spp=1, max_depth=4, mode="mega", flags=ptmi.FLAG_PROFILE)
    assert e.value.code == ptmi.PT_EINVAL
    # more traversal spill area than the scratch holds
    with pytest.raises(ptmi.PtError) as e:
        R.render_noalloc(spp=1, max_depth=4, grid_mult=64, stack_lds=8)
    assert e.value.code == ptmi.PT_ENOMEM
    # the wavefront needs a workspace
    a = R.args(spp=1, max_depth=4, mode="wave")
    out = torch.empty((48, 64, 3), device="cuda")
    rc = ptmi.lib().pt_render_frame_noalloc(R.h, ptmi.C.byref(a), out.data_ptr(), None, R._stream())
    assert rc == ptmi.PT_EUNSUPPORTED
