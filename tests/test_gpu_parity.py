"""GPU parity: the HIP megakernel and wavefront (through the C ABI) against
the CPU oracle, element by element on the same seeded inputs.

Bar (per pixel, all channels): |g - o| <= 1e-4 max(|g|, |o|) + 1e-6 mean(o)
on at least 99.9% of pixels, every failing pixel flagged fragile by the
oracle (a float decision within rounding distance of flipping).  The two
schedules must agree bit for bit with each other.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2605_27323_amd import scenes
from tests._parity import assert_parity, image_tolerance_report

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2605_27323_amd import ptmi  # noqa: E402


def log(*a):
    print(*a, flush=True)


def render_both(R, **kw):
    mega = R.render(mode="mega", **kw).cpu().numpy()
    wave = R.render(mode="wave", **kw).cpu().numpy()
    torch.cuda.synchronize()
    return mega, wave


def test_cornell_full_image_mega_wave_vs_oracle():
    scene, cam = scenes.cornell()
    log("cornell 128x128 spp4 D5 nee")
    R = ptmi.Renderer(scene, cam)
    mega, wave = render_both(R, spp=4, max_depth=5, seed=0)
    assert np.array_equal(mega.view(np.uint32), wave.view(np.uint32))
    S = oracle.Scene(scene)
    ref, frag = S.render(cam, spp=4, max_depth=5, seed=0)
    nexact = assert_parity(wave, ref, frag, what="cornell")
    assert nexact >= 0.999 * ref.shape[0]


@pytest.mark.parametrize("a,D", [(0.5, 3), (0.9, 8)])
def test_white_furnace_exact(a, D):
    le = 1.5
    scene, cam = scenes.furnace(albedo=a, le=le, n=2, width=19, height=13)
    log("furnace", a, D)
    R = ptmi.Renderer(scene, cam)
    mega, wave = render_both(R, spp=2, max_depth=D, seed=3, nee=False)
    af = float(np.float32(a))
    expect = le * sum(af ** k for k in range(D + 1))
    for img in (mega, wave):
        assert np.abs(img - expect).max() <= (2 * D + 6) * 2.0 ** -24 * expect


def test_plane_under_sky_exact():
    scene, cam = scenes.plane_under_sky(albedo=0.6, sky=1.25, width=37, height=23)
    log("plane under sky")
    R = ptmi.Renderer(scene, cam)
    S = oracle.Scene(scene)
    for D in (0, 1, 2):
        mega, wave = render_both(R, spp=1, max_depth=D, seed=1)
        ref, frag = S.render(cam, spp=1, max_depth=D, seed=1)
        assert np.array_equal(wave.reshape(-1, 3), ref)
        assert np.array_equal(mega.reshape(-1, 3), ref)


@pytest.mark.parametrize("cfg", [
    dict(spp=3, max_depth=8, rr_start=3, nee=True, seed=7, frame=0),
    dict(spp=1, max_depth=4, rr_start=-1, nee=False, seed=11, frame=2),
    dict(spp=2, max_depth=0, rr_start=-1, nee=True, seed=5, frame=1),
])
def test_procedural_small_all_pixels(cfg):
    scene, cam = scenes.procedural(seed=21, n_objects=40, width=97, height=61)
    log("procedural 40 objects", scene["indices"].shape[0], "tris", cfg)
    R = ptmi.Renderer(scene, cam)
    mega, wave = render_both(R, **cfg)
    assert np.array_equal(mega.view(np.uint32), wave.view(np.uint32))
    S = oracle.Scene(scene)
    ref, frag = S.render(cam, **cfg)
    assert_parity(wave, ref, frag, what=f"procedural {cfg}")


def test_divergence_materials_with_dielectrics():
    scene, cam = scenes.procedural(seed=31, n_objects=60, width=80, height=48, material_mode="divergence")
    log("divergence 60 objects", scene["indices"].shape[0])
    R = ptmi.Renderer(scene, cam)
    cfg = dict(spp=2, max_depth=12, rr_start=3, nee=True, seed=9)
    mega, wave = render_both(R, **cfg)
    assert np.array_equal(mega.view(np.uint32), wave.view(np.uint32))
    srt = R.render(mode="wave", flags=ptmi.FLAG_SORT_MATERIAL, **cfg).cpu().numpy()
    assert np.array_equal(srt.view(np.uint32), wave.view(np.uint32))
    S = oracle.Scene(scene)
    ref, frag = S.render(cam, **cfg)
    assert_parity(wave, ref, frag, what="divergence")


def test_full_size_procedural_sampled_pixels():
    # the benchmark workload: ~1M triangles, 1920x1080, 1 spp, depth 8, roulette from 3
    scene, cam = scenes.procedural(seed=2, n_objects=2000)
    log("procedural 1M", scene["indices"].shape[0], "tris 1920x1080")
    R = ptmi.Renderer(scene, cam)
    S = oracle.Scene(scene)
    px = scenes.pixel_subset(1920, 1080, 16384, seed=1234)
    for frame in (0, 5):
        cfg = dict(spp=1, max_depth=8, rr_start=3, nee=True, seed=0, frame=frame)
        mega, wave = render_both(R, **cfg)
        assert np.array_equal(mega.view(np.uint32), wave.view(np.uint32))
        ref, frag = S.render(cam, pixels=px, **cfg)
        assert_parity(wave.reshape(-1, 3)[px], ref, frag, what=f"1M frame {frame}")
        # the launch configurations the benchmark times: frame by frame, and
        # frames in flight (the last frame of a run ending at `frame`)
        tuned = R.render(mode="wave", block=256, grid_mult=8, stack_lds=8, tail_threshold=1 << 18, tail_bounce=4,
                         **cfg)
        assert np.array_equal(tuned.cpu().numpy().view(np.uint32), wave.view(np.uint32))
        spread = R.render(mode="wave", block=256, grid_mult=8, stack_lds=8, tail_threshold=1 << 18, tail_bounce=3,
                          tail_spread=True, **cfg)
        assert np.array_equal(spread.cpu().numpy().view(np.uint32), wave.view(np.uint32))
        kw = {k: v for k, v in cfg.items() if k != "frame"}
        inflight = R.render_frames(3, mode="wave", frame=frame - 2 if frame >= 2 else 0, block=256, grid_mult=4,
                                   stack_lds=8, tail_threshold=1 << 18, tail_bounce=3, **kw)
        if frame >= 2:
            assert np.array_equal(inflight.cpu().numpy().view(np.uint32), wave.view(np.uint32))


def test_edge_cases():
    log("edge cases")
    # empty scene: every pixel sees the sky
    base = scenes.random_soup(3, 4)
    empty = dict(base, indices=np.zeros((0, 3), np.int32), tri_mat=np.zeros(0, np.int32),
                 albedo=np.zeros((0, 3), np.float32), emission=np.zeros((0, 3), np.float32),
                 sky=np.array([0.25, 0.5, 1.0], np.float32))
    cam = dict(eye=(0, 0, -3.0), target=(0, 0, 0), up=(0, 1, 0), vfov_deg=45.0, width=5, height=3)
    R = ptmi.Renderer(empty, cam)
    mega, wave = render_both(R, spp=2, max_depth=3)
    assert (mega == empty["sky"]).all() and (wave == empty["sky"]).all()
    # single pixel, single triangle, no lights
    one = scenes.random_soup(4, 1, emissive_frac=0.0)
    one["sky"] = np.array([1.0, 1.0, 1.0], np.float32)
    cam1 = dict(eye=(0, 0, -3.0), target=(0, 0, 0), up=(0, 1, 0), vfov_deg=60.0, width=1, height=1)
    R1 = ptmi.Renderer(one, cam1)
    S1 = oracle.Scene(one)
    for spp in (1, 5):
        mega, wave = render_both(R1, spp=spp, max_depth=2)
        ref, _ = S1.render(cam1, spp=spp, max_depth=2)
        assert np.array_equal(wave.reshape(-1, 3), ref) and np.array_equal(mega.reshape(-1, 3), ref)


@pytest.mark.parametrize("only_degenerate_lights", [False, True])
def test_degenerate_triangles(only_degenerate_lights):
    from tests._parity import degenerate_scene
    scene, cam = degenerate_scene(only_degenerate_lights)
    log("degenerate triangles", only_degenerate_lights)
    R = ptmi.Renderer(scene, cam)
    mega, wave = render_both(R, spp=4, max_depth=5, seed=0)
    assert np.array_equal(mega.view(np.uint32), wave.view(np.uint32))
    assert np.isfinite(wave).all()
    ref, frag = oracle.Scene(scene).render(cam, spp=4, max_depth=5, seed=0)
    nexact = assert_parity(wave.reshape(-1, 3), ref, frag, what="degenerate")
    assert nexact == ref.shape[0]


def test_no_compaction_and_launch_shapes_bit_identical():
    scene, cam = scenes.procedural(seed=41, n_objects=30, width=64, height=40)
    log("launch shapes")
    R = ptmi.Renderer(scene, cam)
    cfg = dict(spp=2, max_depth=6, rr_start=2, seed=3)
    ref = R.render(mode="wave", **cfg).cpu().numpy()
    outs = [R.render(mode="wave", flags=ptmi.FLAG_NO_COMPACT, **cfg),
            R.render(mode="wave", block=64, grid_mult=1, **cfg),
            R.render(mode="wave", block=256, grid_mult=3, **cfg),
            R.render(mode="mega", block=64, grid_mult=2, **cfg),
            R.render(mode="mega", mega_waves=5, **cfg),
            R.render(mode="wave", flags=ptmi.FLAG_SORT_MATERIAL, **cfg),
            R.render(mode="wave", flags=ptmi.FLAG_SORT_MATERIAL, sort_threshold=1500, **cfg),
            R.render(mode="wave", flags=ptmi.FLAG_SORT_MATERIAL, block=64, grid_mult=1, **cfg),
            R.render(mode="wave", tail_threshold=700, **cfg),
            R.render(mode="wave", tail_threshold=1 << 30, stack_lds=8, **cfg),
            R.render(mode="wave", tail_threshold=300, flags=ptmi.FLAG_SORT_MATERIAL, **cfg),
            R.render(mode="wave", flags=ptmi.FLAG_SORT_RAYS, **cfg),
            R.render(mode="wave", flags=ptmi.FLAG_SORT_RAYS | ptmi.FLAG_SORT_MATERIAL, sort_threshold=900,
                     tail_threshold=200, **cfg),
            R.render(mode="wave", tail_bounce=1, **cfg),
            R.render(mode="wave", tail_bounce=3, tail_threshold=300, **cfg),
            R.render(mode="wave", tail_bounce=6, flags=ptmi.FLAG_SORT_MATERIAL, **cfg),
            R.render(mode="wave", tail_bounce=2, tail_spread=True, **cfg),
            R.render(mode="wave", tail_threshold=1 << 30, tail_spread=True, block=64, grid_mult=1, **cfg),
            R.render(mode="wave", tail_threshold=500, tail_spread=True, flags=ptmi.FLAG_SORT_MATERIAL, **cfg),
            R.render(mode="wave", flags=ptmi.FLAG_XCD_LOCAL, **cfg),
            R.render(mode="wave", flags=ptmi.FLAG_XCD_LOCAL, block=64, grid_mult=3, tail_bounce=3, **cfg),
            R.render(mode="mega", flags=ptmi.FLAG_XCD_LOCAL, **cfg),
            R.render(mode="mega", flags=ptmi.FLAG_XCD_LOCAL, block=128, grid_mult=1, mega_waves=5, **cfg),
            R.render(mode="wave", **cfg)]
    # the image does not depend on the BVH either: leaves of up to 4 and 8 triangles
    for ml in (4, 8):
        Rl = ptmi.Renderer(scene, cam, max_leaf=ml)
        outs += [Rl.render(mode="wave", **cfg), Rl.render(mode="mega", **cfg)]
    for o in outs:
        assert np.array_equal(o.cpu().numpy().view(np.uint32), ref.view(np.uint32))


def test_progressive_accumulation_and_ray_counts():
    scene, cam = scenes.cornell()
    cam = dict(cam, width=33, height=17)
    log("progressive")
    R = ptmi.Renderer(scene, cam)
    S = oracle.Scene(scene)
    acc = torch.zeros((17, 33, 3), dtype=torch.float32, device="cuda")
    ref_acc = None
    for frame in range(4):
        R.render(mode="wave" if frame % 2 else "mega", accum=acc, spp=2, max_depth=4, frame=frame)
        I, _ = S.render(cam, spp=2, max_depth=4, frame=frame)
        if ref_acc is None:
            ref_acc = I.copy()
        else:
            n = np.float32(frame + 1)
            ref_acc = (ref_acc + (I - ref_acc) / n).astype(np.float32)
    got = acc.cpu().numpy().reshape(-1, 3)
    frac, nfail, unexplained, nexact = image_tolerance_report(got, ref_acc, np.zeros(len(ref_acc)))
    assert nexact >= 0.999 * len(ref_acc)
    # identical paths => identical ray counts in both schedules
    R.render(mode="mega", spp=2, max_depth=4, flags=ptmi.FLAG_COUNT_WORK)
    sm = R.stats()
    R.render(mode="wave", spp=2, max_depth=4, flags=ptmi.FLAG_COUNT_WORK)
    sw = R.stats()
    assert sm["extension_rays"] == sw["extension_rays"] > 0
    assert sm["shadow_rays"] == sw["shadow_rays"] > 0
    # every ray is traversed identically in both schedules: same node visits
    # and triangle tests in total
    for key in ("node_visits", "tri_tests"):
        assert sm[key]["mega"] == sw[key]["extend"] + sw[key]["shadow"] > 0
    # the hybrid tail traces the rest of the paths in place and counts them
    R.render(mode="wave", spp=2, max_depth=4, tail_threshold=400, flags=ptmi.FLAG_COUNT_WORK)
    st = R.stats()
    assert st["items"].get("tail", 0) > 0
    assert (st["extension_rays"], st["shadow_rays"]) == (sm["extension_rays"], sm["shadow_rays"])
    for key in ("node_visits", "tri_tests"):
        assert sum(st[key].values()) == sm[key]["mega"]
    # the same with the tail taking over at bounce 2
    R.render(mode="wave", spp=2, max_depth=4, tail_bounce=2, flags=ptmi.FLAG_COUNT_WORK)
    sb = R.stats()
    assert sb["items"].get("tail", 0) > 0
    assert (sb["extension_rays"], sb["shadow_rays"]) == (sm["extension_rays"], sm["shadow_rays"])
    for key in ("node_visits", "tri_tests"):
        assert sum(sb[key].values()) == sm[key]["mega"]


def test_profile_stage_times():
    scene, cam = scenes.procedural(seed=51, n_objects=20, width=48, height=32)
    R = ptmi.Renderer(scene, cam)
    R.render(mode="wave", spp=1, max_depth=5, rr_start=3, flags=ptmi.FLAG_PROFILE)
    st = R.stats()
    assert st["launches"]["extend"] == 6 and st["launches"]["shade"] == 6
    assert all(v >= 0 for v in st["stage_ms"].values())
    # work items and algorithmic bytes follow from the queue counts
    it, by = st["items"], st["bytes"]
    assert it["raygen"] == 48 * 32 and it["accumulate"] == 48 * 32
    assert it["extend"] == st["extension_rays"] and it["shadow"] == st["shadow_rays"]
    assert it["shade"] == it["extend"] and "tail" not in it
    assert by["extend"] == 48 * it["extend"] and by["shadow"] == 48 * it["shadow"]
    assert by["shade"] == 80 * it["shade"] + 48 * (it["extend"] - it["raygen"]) + 48 * it["shadow"]
    R.render(mode="wave", spp=1, max_depth=5, rr_start=3, tail_threshold=1 << 30, flags=ptmi.FLAG_PROFILE)
    st = R.stats()
    assert st["launches"]["tail"] == 6 and st["items"]["tail"] == 48 * 32 and "shade" not in st["items"]
    # tail_bounce: no stage of a later bounce is launched
    R.render(mode="wave", spp=1, max_depth=5, rr_start=3, tail_bounce=2, flags=ptmi.FLAG_PROFILE)
    st = R.stats()
    assert st["launches"]["extend"] == 3 and st["launches"]["tail"] == 1 and st["launches"]["shadow"] == 2


def _frames_ws(R, **kw):
    n = ctypes.c_uint64()
    assert ptmi.lib().pt_frames_workspace_size(R.h, ctypes.byref(R.args(**kw)), ctypes.byref(n)) == 0
    return n.value


@pytest.mark.parametrize("queues", ["4", "8", "10"])
@pytest.mark.parametrize("mode", ["wave", "mega"])
def test_frames_in_flight_match_sequential(mode, queues, monkeypatch):
    """pt_render_frames (three frames in flight on internal streams, six
    when the process has eight hardware queues, eight with ten) gives the
    same running average and last image, bit for bit, as frame-by-frame
    rendering."""
    scene, cam = scenes.procedural(seed=52, n_objects=30, width=64, height=40)
    log(f"frames in flight {mode}, {queues} queues")
    monkeypatch.setenv("GPU_MAX_HW_QUEUES", queues)
    R = ptmi.Renderer(scene, cam)  # the count of frames in flight is fixed here
    monkeypatch.setenv("GPU_MAX_HW_QUEUES", "4")
    R4 = ptmi.Renderer(scene, cam)
    kw = dict(mode=mode, spp=2, max_depth=6, rr_start=3, tail_threshold=300 if mode == "wave" else 0,
              tail_bounce=4 if mode == "wave" else 0)
    # three, six or eight frame slots
    assert _frames_ws(R, **kw) * 3 == _frames_ws(R4, **kw) * {"4": 3, "8": 6, "10": 8}[queues]
    acc_seq = torch.zeros((40, 64, 3), dtype=torch.float32, device="cuda")
    for f in range(5):
        img_seq = R.render(accum=acc_seq, frame=3 + f, **kw).clone()
    # continue the same running average both ways from frame 8, over more
    # frames than there are slots
    acc_pipe = acc_seq.clone()
    acc_seq2 = acc_seq.clone()
    for f in range(9):
        R.render(accum=acc_seq2, frame=8 + f, **kw)
    img_pipe = R.render_frames(9, accum=acc_pipe, frame=8, **kw)
    torch.cuda.synchronize()
    assert torch.equal(acc_pipe.view(torch.int32), acc_seq2.view(torch.int32))
    img_last = R.render(frame=16, **kw)
    assert torch.equal(img_pipe.view(torch.int32), img_last.view(torch.int32))
    # one frame through the pipelined entry point equals a plain frame
    one = R.render_frames(1, frame=0, **kw).clone()
    assert torch.equal(one.view(torch.int32), R.render(frame=0, **kw).view(torch.int32))


def test_halton_sampler_vs_oracle():
    """sampler="halton" (Halton(2,3) camera jitter with a per-pixel rotation):
    the same bar against the oracle's sampler; mega = wave bit for bit; frames
    in flight equal frame-by-frame rendering."""
    scene, cam = scenes.procedural(seed=24, n_objects=40, width=97, height=61)
    log("halton sampler 97x61 spp 6")
    R = ptmi.Renderer(scene, cam)
    cfg = dict(spp=6, max_depth=6, rr_start=3, seed=13, frame=2, sampler="halton")
    mega, wave = render_both(R, **cfg)
    assert np.array_equal(mega.view(np.uint32), wave.view(np.uint32))
    ref, frag = oracle.Scene(scene).render(cam, **dict(cfg, sampler=1))
    nexact = assert_parity(wave, ref, frag, what="halton")
    assert nexact >= 0.99 * ref.shape[0]
    philox = R.render(mode="wave", **dict(cfg, sampler="philox")).cpu().numpy()
    assert not np.array_equal(philox, wave)
    kw = dict(cfg, mode="wave", tail_threshold=300, tail_bounce=4)
    acc_seq = torch.zeros((61, 97, 3), dtype=torch.float32, device="cuda")
    for f in range(3):
        R.render(accum=acc_seq, frame=f, **{k: v for k, v in kw.items() if k != "frame"})
    acc_pipe = torch.zeros_like(acc_seq)
    R.render_frames(3, accum=acc_pipe, **kw | dict(frame=0))
    torch.cuda.synchronize()
    assert torch.equal(acc_pipe.view(torch.int32), acc_seq.view(torch.int32))
    with pytest.raises(ValueError):
        R.render(sampler="sobol")
    a = R.args(spp=1)  # the C ABI rejects other values before any launch
    a.sampler = 2
    ws, wsb = R.workspace(R.args(spp=1))
    out = torch.empty((61, 97, 3), dtype=torch.float32, device="cuda")
    assert ptmi.lib().pt_render_frame(R.h, ctypes.byref(a), out.data_ptr(), None, ws, wsb, R._stream()) == -1
    a = R.args(spp=1)
    a.tail_spread = 2  # 0 or 1 only
    assert ptmi.lib().pt_render_frame(R.h, ctypes.byref(a), out.data_ptr(), None, ws, wsb, R._stream()) == -1


def test_two_slot_count_buffer_bit_identical():
    # the paper's two-slot live count with a promote kernel between bounces
    # (Sec. 3.1), as an ablation of the per-bounce counters: same image and
    # ray counts in every wavefront configuration, one promote per bounce
    scene, cam = scenes.procedural(seed=41, n_objects=30, width=64, height=40)
    log("two-slot counts")
    R = ptmi.Renderer(scene, cam)
    cfg = dict(spp=2, max_depth=6, rr_start=2, seed=3)
    T = ptmi.FLAG_TWO_SLOT
    for kw in (dict(), dict(flags=ptmi.FLAG_NO_COMPACT), dict(flags=ptmi.FLAG_SORT_MATERIAL | ptmi.FLAG_SORT_RAYS),
               dict(tail_threshold=700), dict(tail_bounce=3, tail_threshold=300), dict(block=64, grid_mult=1)):
        flags = kw.pop("flags", 0)
        ref = R.render(mode="wave", flags=flags, **kw, **cfg).cpu().numpy()
        st_ref = R.stats()
        img = R.render(mode="wave", flags=flags | T, **kw, **cfg).cpu().numpy()
        st = R.stats()
        assert np.array_equal(img.view(np.uint32), ref.view(np.uint32)), kw
        assert st["extension_rays"] == st_ref["extension_rays"] and st["shadow_rays"] == st_ref["shadow_rays"], kw
        assert st["items"].get("extend") == st_ref["items"].get("extend"), kw
        assert st["items"]["promote"] >= 2 and "promote" not in st_ref["items"], kw
    # frames in flight
    out_a = torch.zeros((40, 64, 3), device="cuda")
    out_b = torch.zeros((40, 64, 3), device="cuda")
    R.render_frames(4, out=out_a, mode="wave", **cfg)
    R.render_frames(4, out=out_b, mode="wave", flags=T, **cfg)
    torch.cuda.synchronize()
    assert torch.equal(out_a, out_b)


def test_serial_stages_bit_identical():
    # every stage on the render stream (PT_FLAG_SERIAL_STAGES) against the
    # shadow stage beside the next extend stage: same image and ray counts,
    # with and without compaction and the hybrid tail
    scene, cam = scenes.procedural(seed=43, n_objects=30, width=64, height=40)
    log("serial stages")
    R = ptmi.Renderer(scene, cam)
    cfg = dict(spp=2, max_depth=6, rr_start=2, seed=5)
    S = ptmi.FLAG_SERIAL_STAGES
    for kw in (dict(), dict(flags=ptmi.FLAG_NO_COMPACT), dict(tail_bounce=3, tail_threshold=300)):
        flags = kw.pop("flags", 0)
        ref = R.render(mode="wave", flags=flags | S, **kw, **cfg).cpu().numpy()
        st_ref = R.stats()
        img = R.render(mode="wave", flags=flags, **kw, **cfg).cpu().numpy()
        st = R.stats()
        assert np.array_equal(img.view(np.uint32), ref.view(np.uint32)), kw
        assert st["extension_rays"] == st_ref["extension_rays"] and st["shadow_rays"] == st_ref["shadow_rays"], kw
