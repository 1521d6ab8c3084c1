"""The HIP kernels' own arithmetic, compiled for the host (tests/emu), against
the independent CPU oracle: catches logic and indexing errors of the device
code before it runs on a GPU.  The megakernel body runs per pixel; the
wavefront stage items run stage by stage with shuffled queues."""
import numpy as np
import pytest

import oracle
from paper_2605_27323_amd import scenes
from tests._parity import assert_parity

emu = pytest.importorskip("tests.emu")


def _check(scene, cam, pixels=None, **cfg):
    E = emu.Emu(scene, cam)
    img, rays = E.mega(pixels=pixels, **cfg)
    ref, frag = oracle.Scene(scene).render(cam, pixels=pixels, **cfg)
    nexact = assert_parity(img, ref, frag, what=str(cfg))
    return E, img, rays, nexact


def test_cornell_bit_exact_and_wave_equals_mega():
    scene, cam = scenes.cornell()
    cfg = dict(spp=4, max_depth=5, seed=0)
    E, img, rays, nexact = _check(scene, cam, **cfg)
    assert nexact == img.shape[0]
    for shuffle in (0, 5):
        w, rw = E.wave(shuffle=shuffle, **cfg)
        assert np.array_equal(w.view(np.uint32), img.view(np.uint32))
        assert (rw == rays).all()
    w, _ = E.wave(compact=False, **cfg)
    assert np.array_equal(w.view(np.uint32), img.view(np.uint32))


@pytest.mark.parametrize("mode,cfg", [
    ("lambert_conductor", dict(spp=3, max_depth=8, rr_start=3, seed=7, frame=2)),
    ("lambert_conductor", dict(spp=1, max_depth=3, rr_start=-1, nee=False, seed=1)),
    ("divergence", dict(spp=2, max_depth=16, rr_start=3, seed=9)),
])
def test_procedural_scenes(mode, cfg):
    scene, cam = scenes.procedural(seed=21, n_objects=40, width=61, height=37, material_mode=mode)
    E, img, rays, nexact = _check(scene, cam, **cfg)
    assert nexact >= 0.999 * img.shape[0]
    w, rw = E.wave(shuffle=11, **cfg)
    assert np.array_equal(w.view(np.uint32), img.view(np.uint32))
    assert (rw == rays).all()
    w, rw = E.wave(sort=True, shuffle=3, **cfg)
    assert np.array_equal(w.view(np.uint32), img.view(np.uint32))
    for tail in (1, 500, 10 ** 9):  # hybrid tail from some bounce on, or from the start
        w, rt = E.wave(tail=tail, shuffle=tail, **cfg)
        assert np.array_equal(w.view(np.uint32), img.view(np.uint32))
        assert (rt == rays).all()  # the tail's in-place rays are counted too


def test_furnace_and_sky_exact():
    scene, cam = scenes.furnace(albedo=0.9, le=2.0, n=3, width=9, height=7)
    E = emu.Emu(scene, cam)
    img, _ = E.mega(spp=2, max_depth=10, nee=False)
    expect = 2.0 * sum(float(np.float32(0.9)) ** k for k in range(11))
    assert np.abs(img - expect).max() <= 30 * 2.0 ** -24 * expect
    scene, cam = scenes.plane_under_sky(albedo=0.6, sky=1.25, width=21, height=13)
    E = emu.Emu(scene, cam)
    img, _ = E.mega(spp=1, max_depth=2)
    ref, _ = oracle.Scene(scene).render(cam, spp=1, max_depth=2)
    assert np.array_equal(img, ref)


def test_empty_and_single_triangle():
    base = scenes.random_soup(3, 4)
    empty = dict(base, indices=np.zeros((0, 3), np.int32), tri_mat=np.zeros(0, np.int32),
                 albedo=np.zeros((0, 3), np.float32), emission=np.zeros((0, 3), np.float32),
                 sky=np.array([0.25, 0.5, 1.0], np.float32))
    cam = dict(eye=(0, 0, -3.0), target=(0, 0, 0), up=(0, 1, 0), vfov_deg=45.0, width=5, height=3)
    E = emu.Emu(empty, cam)
    img, rays = E.mega(spp=2, max_depth=3)
    assert (img == empty["sky"]).all() and rays[0] == 30
    w, _ = E.wave(spp=2, max_depth=3)
    assert (w == empty["sky"]).all()
    one = scenes.random_soup(4, 1, emissive_frac=1.0)
    cam = dict(eye=(0, 0, -3.0), target=(0, 0, 0), up=(0, 1, 0), vfov_deg=70.0, width=8, height=8)
    _check(one, cam, spp=3, max_depth=2)


@pytest.mark.parametrize("max_leaf", [2, 4, 8])
def test_leaf_sizes_give_the_same_image(max_leaf):
    # multi-triangle leaves (the leaf loop) against the default of one
    # triangle per leaf: the image does not depend on the BVH
    scene, cam = scenes.procedural(seed=5, n_objects=40, width=40, height=24)
    cfg = dict(spp=2, max_depth=6, rr_start=2, seed=4)
    ref, _ = emu.Emu(scene, cam).mega(**cfg)
    E = emu.Emu(scene, cam, max_leaf=max_leaf)
    for img in (E.mega(**cfg)[0], E.wave(shuffle=3, **cfg)[0]):
        assert np.array_equal(img.view(np.uint32), ref.view(np.uint32))
    o = scenes.random_soup(13, 300)
    d = np.random.default_rng(max_leaf).normal(size=(400, 3)).astype(np.float32)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    org = np.zeros((400, 3), np.float32)
    a = emu.Emu(o, cam).closest(org, d)
    b = emu.Emu(o, cam, max_leaf=max_leaf).closest(org, d)
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32))


def test_rays_in_all_octants_never_touch_empty_slots():
    # nodes with fewer than four children keep +inf boxes in the free slots;
    # rays with every direction component positive used to accept them
    scene = scenes.random_soup(8, 7, emissive_frac=0.3)
    for eye in [(-3.0, -3.0, -3.0), (3.0, 3.0, 3.0), (-3.0, 3.0, -3.0), (3.0, -3.0, 3.0)]:
        cam = dict(eye=eye, target=(0, 0, 0), up=(0, 1, 0), vfov_deg=60.0, width=12, height=12)
        _check(scene, cam, spp=2, max_depth=4)


@pytest.mark.parametrize("dist,offset", [(1.0, 0.0), (30.0, 0.0), (1e3, 0.0), (1e5, 0.0), (0.5, 3e4), (5.0, -1e6)])
def test_closest_hit_from_distant_origins_equals_brute_force(dist, offset):
    # rays aimed at vertices and edge points (where a hit sits on the boundary
    # of its leaf box) from origins up to 1e5 times the scene's extent, and
    # from nearby origins in a scene far from the coordinate origin (large
    # coordinates, short distances): the slab test must stay conservative,
    # so the closest hit equals the oracle's brute force bit for bit
    scene = scenes.random_soup(12, 80, emissive_frac=0.1)
    scene = dict(scene, positions=(scene["positions"] + np.float32(offset)).astype(np.float32))
    cam = dict(eye=(0, 0, -3.0), target=(0, 0, 0), up=(0, 1, 0), vfov_deg=45.0, width=4, height=4)
    E = emu.Emu(scene, cam)
    rng = np.random.default_rng(int(dist))
    pos, idx = scene["positions"], scene["indices"]
    v = pos[idx]  # [nt, 3, 3]
    w = rng.dirichlet([0.2, 0.2, 0.2], size=(600,)).astype(np.float32)
    w[:200] = np.eye(3, dtype=np.float32)[rng.integers(0, 3, 200)]  # vertices
    w[200:400, rng.integers(0, 3)] = 0.0  # edges
    w[200:400] /= w[200:400].sum(1, keepdims=True)
    tri = rng.integers(0, idx.shape[0], 600)
    target = np.einsum("nk,nkc->nc", w, v[tri]).astype(np.float32)
    u = rng.normal(size=(600, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    u[::7] = np.eye(3)[rng.integers(0, 3, len(u[::7]))] * rng.choice([-1, 1], (len(u[::7]), 1))  # axis-parallel
    o = (target - dist * u).astype(np.float32)
    assert not np.array_equal(o, target)
    d = (target - o).astype(np.float64)
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    t, i, b1, b2 = E.closest(o, d)
    rt, ri, rb1, rb2 = oracle.Scene(scene).closest(o, d, mode=0)
    assert (ri >= 0).mean() > 0.5
    assert np.array_equal(i, ri)
    hit = ri >= 0
    for a, r in [(t, rt), (b1, rb1), (b2, rb2)]:
        assert np.array_equal(a[hit].view(np.uint32), r[hit].view(np.uint32))


def test_full_size_scene_sampled_pixels():
    scene, cam = scenes.procedural(seed=2, n_objects=2000)
    px = scenes.pixel_subset(1920, 1080, 4096, seed=99)
    E, img, rays, nexact = _check(scene, cam, pixels=px, spp=1, max_depth=8, rr_start=3, seed=0, frame=1)
    assert nexact >= 0.999 * len(px)


@pytest.mark.parametrize("which", ["cornell", "conductor"])
def test_adjoint_matches_oracle(which):
    scene, cam = scenes.cornell()
    cam = dict(cam, width=24, height=20)
    if which == "conductor":
        scene = {k: v.copy() for k, v in scene.items()}
        scene["materials"] = np.array([[0, 1.0, 1.5, 0], [1, 0.35, 1.5, 0]], np.float32)
        scene["tri_mat"][10:22] = 1
    E = emu.Emu(scene, cam)
    rng = np.random.default_rng(0)
    d = rng.normal(size=(cam["width"] * cam["height"], 3)).astype(np.float32)
    ga, ge = E.backward(d, spp=2, max_depth=4, seed=3)
    oa, oe, aa, ae = oracle.Scene(scene).backward(cam, d, spp=2, max_depth=4, seed=3)
    for g, o, a in [(ga, oa, aa), (ge, oe, ae)]:
        # per entry: 1e-4 of the summed absolute terms plus 1e-7 of the largest gradient
        assert (np.abs(g - o) <= 1e-4 * a + 1e-7 * np.abs(o).max()).all()
        assert np.linalg.norm(g - o) <= 1e-4 * np.linalg.norm(o)


@pytest.mark.parametrize("capacity", [64, 333, 100000])
def test_batch_pool_equals_standalone(capacity):
    jobs, scenes_ = [], []
    for j, (seed, n, w, h, spp) in enumerate([(1000, 8, 33, 21, 2), (1001, 20, 16, 16, 3), (1002, 3, 40, 8, 1)]):
        s, c = scenes.procedural(seed=seed, n_objects=n, width=w, height=h)
        jobs.append((emu.Emu(s, c), dict(spp=spp, max_depth=6, rr_start=3, seed=5, frame=1)))
        scenes_.append((s, c))
    imgs, it = emu.render_batch([e for e, _ in jobs], [kw for _, kw in jobs], capacity, shuffle=capacity)
    for j, (e, kw) in enumerate(jobs):
        ref, _ = e.mega(job=j, **kw)
        assert np.array_equal(imgs[j].view(np.uint32), ref.view(np.uint32))
        # the oracle's image of job j (the job index keys its random numbers)
        o, frag = oracle.Scene(scenes_[j][0]).render(scenes_[j][1], job=j, **kw)
        assert_parity(imgs[j], o, frag, what=f"pool job {j}")


def test_far_camera():
    # a camera far outside the scene (slab distances from large origins)
    scene = scenes.random_soup(9, 60, emissive_frac=0.2)
    for dist in (5.0, 400.0):
        cam = dict(eye=(0.3 * dist, 0.2 * dist, -dist), target=(0, 0, 0), up=(0, 1, 0),
                   vfov_deg=60.0 * 5.0 / dist, width=16, height=12)
        _check(scene, cam, spp=2, max_depth=4)


def test_halton_sampler_matches_oracle():
    # the device code's radical inverses and rotation against the oracle's:
    # same camera rays, so the same images bit for bit; wave = mega; the
    # adjoint replays the same camera rays; the batch pool carries the sampler
    scene, cam = scenes.procedural(seed=23, n_objects=30, width=45, height=29)
    cfg = dict(spp=6, max_depth=5, rr_start=3, seed=3, frame=7, sampler=1)
    E, img, rays, nexact = _check(scene, cam, **cfg)
    assert nexact >= 0.999 * img.shape[0]
    philox, _ = E.mega(**dict(cfg, sampler=0))
    assert not np.array_equal(img, philox)
    w, rw = E.wave(shuffle=4, tail=300, **cfg)
    assert np.array_equal(w.view(np.uint32), img.view(np.uint32))
    assert (rw == rays).all()
    rng = np.random.default_rng(1)
    d = rng.normal(size=(cam["width"] * cam["height"], 3)).astype(np.float32)
    ga, ge = E.backward(d, spp=2, max_depth=4, seed=3, sampler=1)
    oa, oe, aa, ae = oracle.Scene(scene).backward(cam, d, spp=2, max_depth=4, seed=3, sampler=1)
    for g, o, a in [(ga, oa, aa), (ge, oe, ae)]:
        assert (np.abs(g - o) <= 1e-4 * a + 1e-7 * np.abs(o).max()).all()
    imgs, _ = emu.render_batch([E], [dict(cfg, job=0)], 500, shuffle=2)
    assert np.array_equal(imgs[0].view(np.uint32), E.mega(**cfg)[0].view(np.uint32))


@pytest.mark.parametrize("only_degenerate_lights", [False, True])
def test_degenerate_triangles(only_degenerate_lights):
    # zero-area triangles, emissive ones among them: never hit, never picked
    # as a light sample (zero area), no NaN; with no light of positive area
    # the sky alone lights the box
    from tests._parity import degenerate_scene
    scene, cam = degenerate_scene(only_degenerate_lights)
    E, img, rays, nexact = _check(scene, cam, spp=4, max_depth=5, seed=0)
    assert np.isfinite(img).all() and nexact == img.shape[0]
    w, _ = E.wave(shuffle=3, spp=4, max_depth=5, seed=0)
    assert np.array_equal(w.view(np.uint32), img.view(np.uint32))


def test_instanced_scene_matches_oracle():
    # two-level scene: the library's instanced traversal and shading (device
    # code on the host) against the oracle's instanced path loop; wavefront
    # with shuffled queues and the hybrid tail = megakernel
    sc, inst, cam = scenes.instanced_procedural(seed=9, n_instances=80, n_meshes=8, width=40, height=28)
    E = emu.Emu(sc, cam, instances=inst)
    S = oracle.Scene(sc, instances=inst)
    for cfg in (dict(spp=2, max_depth=6, rr_start=3, seed=5, frame=1), dict(spp=1, max_depth=3, nee=False, seed=2)):
        img, rays = E.mega(**cfg)
        o, frag = S.render(cam, **cfg)
        nexact = assert_parity(img, o, frag, what=f"instanced {cfg}")
        assert nexact >= 0.999 * img.shape[0]
        w, rw = E.wave(shuffle=3, tail=200, **cfg)
        assert np.array_equal(w.view(np.uint32), img.view(np.uint32)) and (rw == rays).all()


def test_identity_instances_equal_flat_scene():
    sc, cam = scenes.procedural(seed=21, n_objects=30, width=40, height=28)
    cfg = dict(spp=2, max_depth=6, rr_start=3, seed=5, frame=1)
    a, _ = emu.Emu(sc, cam).mega(**cfg)
    for parts in (1, 5):
        b, _ = emu.Emu(sc, cam, instances=scenes.split_into_instances(sc, parts)).mega(**cfg)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), parts


@pytest.mark.parametrize("cfg", [dict(spp=3, max_depth=6, rr_start=3, seed=4, frame=1),
                                 dict(spp=2, max_depth=4, nee=False, seed=8)])
def test_attributes_match_oracle(cfg):
    # shading normals, checker texture and the coated material: the device
    # shading code against the oracle; wavefront (shuffled, sorted, hybrid
    # tail) = megakernel bit for bit
    scene, cam = scenes.cornell_attributes(coat=(0.3, 1.5))
    cam = dict(cam, width=40, height=32)
    E, img, rays, nexact = _check(scene, cam, **cfg)
    assert nexact >= 0.999 * img.shape[0]
    for kw in (dict(shuffle=7), dict(sort=True, shuffle=2), dict(tail=300, shuffle=5)):
        w, rw = E.wave(**kw, **cfg)
        assert np.array_equal(w.view(np.uint32), img.view(np.uint32)), kw
        assert (rw == rays).all()


def test_procedural_attributes_match_oracle():
    scene, cam = scenes.procedural(seed=21, n_objects=40, width=61, height=37, attributes=True)
    assert (scene["materials"][:, 0] == scenes.COATED).any() and (scene["materials"][:, 3] > 0).any()
    cfg = dict(spp=2, max_depth=8, rr_start=3, seed=7, frame=2)
    E, img, rays, nexact = _check(scene, cam, **cfg)
    assert nexact >= 0.999 * img.shape[0]
    w, rw = E.wave(shuffle=9, tail=400, **cfg)
    assert np.array_equal(w.view(np.uint32), img.view(np.uint32))
    # without the attributes the same geometry renders differently
    plain = {k: v for k, v in scene.items() if k not in ("normals", "uvs")}
    p, _ = emu.Emu(plain, cam).mega(**cfg)
    assert not np.array_equal(p, img)


def test_instanced_attributes_match_oracle():
    # smooth-shaded, textured and coated meshes placed by instances: object
    # space normals mapped by the inverse transpose
    sc, inst, cam = scenes.instanced_procedural(seed=9, n_instances=80, n_meshes=8, width=40, height=28,
                                                attributes=True)
    E = emu.Emu(sc, cam, instances=inst)
    S = oracle.Scene(sc, instances=inst)
    cfg = dict(spp=2, max_depth=6, rr_start=3, seed=5, frame=1)
    img, rays = E.mega(**cfg)
    o, frag = S.render(cam, **cfg)
    nexact = assert_parity(img, o, frag, what="instanced attributes")
    assert nexact >= 0.999 * img.shape[0]
    w, rw = E.wave(shuffle=3, tail=200, **cfg)
    assert np.array_equal(w.view(np.uint32), img.view(np.uint32)) and (rw == rays).all()


def test_adjoint_with_attributes_matches_oracle():
    scene, cam = scenes.cornell_attributes(coat=(0.3, 1.5))
    cam = dict(cam, width=24, height=20)
    E = emu.Emu(scene, cam)
    rng = np.random.default_rng(1)
    d = rng.normal(size=(cam["width"] * cam["height"], 3)).astype(np.float32)
    ga, ge = E.backward(d, spp=2, max_depth=4, seed=3)
    oa, oe, aa, ae = oracle.Scene(scene).backward(cam, d, spp=2, max_depth=4, seed=3)
    for g, o, a in [(ga, oa, aa), (ge, oe, ae)]:
        assert (np.abs(g - o) <= 1e-4 * a + 1e-7 * np.abs(o).max()).all()
        assert np.linalg.norm(g - o) <= 1e-4 * np.linalg.norm(o)
    # coated and textured triangles receive albedo gradients
    assert np.abs(oa[scene["tri_mat"] == 1]).sum() > 0 and np.abs(oa[:2]).sum() > 0


@pytest.mark.parametrize("which", ["cornell_attributes", "procedural", "depth0"])
def test_adjoint_keep_hits_bit_identical(which):
    # replay B from replay A's kept intersections and visibilities (no
    # tracing) adds the same terms in the same order: the gradients equal
    # those of the tracing replay bit for bit, and the oracle's
    kw = dict(spp=2, max_depth=4, seed=3, frame=1)
    if which == "cornell_attributes":
        scene, cam = scenes.cornell_attributes(coat=(0.3, 1.5))
        cam = dict(cam, width=20, height=16)
    else:
        scene, cam = scenes.procedural(seed=71, n_objects=25, width=24, height=16)
        if which == "depth0":
            kw["max_depth"] = 0
    E = emu.Emu(scene, cam)
    d = np.random.default_rng(5).normal(size=(cam["width"] * cam["height"], 3)).astype(np.float32)
    ga, ge = E.backward(d, **kw)
    oa, oe, aa, ae = oracle.Scene(scene).backward(cam, d, **kw)
    assert np.abs(oe).sum() > 0
    # 1: replay A path by path; 2: replay A as the wavefront (shuffled
    # queues), its records written by the stage functions; 3: the same with
    # every path finished by the hybrid tail
    for keep in (1, 2, 3):
        ka, ke = E.backward(d, keep_hits=keep, **kw)
        assert np.array_equal(ga.view(np.uint32), ka.view(np.uint32)), keep
        assert np.array_equal(ge.view(np.uint32), ke.view(np.uint32)), keep
        for g, o, a in [(ka, oa, aa), (ke, oe, ae)]:
            assert (np.abs(g - o) <= 1e-4 * a + 1e-7 * np.abs(o).max()).all()


def test_batch_with_attribute_job_matches_oracle():
    s0, c0 = scenes.cornell_attributes(coat=(0.2, 1.4))
    c0 = dict(c0, width=20, height=16)
    s1, c1 = scenes.procedural(seed=1001, n_objects=12, width=16, height=16)
    jobs = [(emu.Emu(s0, c0), dict(spp=2, max_depth=5, rr_start=3, seed=5, frame=1)),
            (emu.Emu(s1, c1), dict(spp=1, max_depth=5, rr_start=3, seed=6))]
    imgs, _ = emu.render_batch([e for e, _ in jobs], [kw for _, kw in jobs], 200, shuffle=4)
    for j, ((s, c), (e, kw)) in enumerate(zip([(s0, c0), (s1, c1)], jobs)):
        o, frag = oracle.Scene(s).render(c, job=j, **kw)
        assert_parity(imgs[j], o, frag, what=f"attribute batch job {j}")


def test_coat_without_attributes_matches_oracle():
    # coated materials alone select the extended shading variant
    scene, cam = scenes.cornell()
    scene = {k: v.copy() for k, v in scene.items()}
    scene["materials"] = np.array([[0, 1.0, 1.5, 0], [scenes.COATED, 0.2, 1.6, 0]], np.float32)
    scene["tri_mat"][10:22] = 1
    cam = dict(cam, width=40, height=32)
    cfg = dict(spp=3, max_depth=6, rr_start=3, seed=4)
    E, img, rays, nexact = _check(scene, cam, **cfg)
    assert nexact >= 0.999 * img.shape[0]
    w, rw = E.wave(shuffle=6, tail=300, **cfg)
    assert np.array_equal(w.view(np.uint32), img.view(np.uint32))


def test_degenerate_triangles_with_attributes():
    # zero-area triangles and random (some zero, some flipped, some huge)
    # vertex normals and texture coordinates with coated and textured
    # materials: finite images equal to the oracle's
    from tests._parity import degenerate_scene
    scene, cam = degenerate_scene(False)
    rng = np.random.default_rng(17)
    nv = scene["positions"].shape[0]
    nrm = rng.normal(size=(nv, 3)) * rng.choice([0.0, 1e-3, 1.0, 1e6], size=(nv, 1))
    scene = dict(scene, normals=nrm.astype(np.float32), uvs=rng.uniform(-50, 50, (nv, 2)).astype(np.float32))
    scene["materials"] = np.array([[0, 1.0, 1.5, 3.0], [scenes.COATED, 0.3, 1.4, 2.0]], np.float32)
    scene["tri_mat"] = (np.arange(scene["indices"].shape[0]) % 2).astype(np.int32)
    E, img, rays, nexact = _check(scene, cam, spp=4, max_depth=5, seed=2)
    assert np.isfinite(img).all() and nexact >= 0.999 * img.shape[0]
    w, _ = E.wave(shuffle=5, spp=4, max_depth=5, seed=2)
    assert np.array_equal(w.view(np.uint32), img.view(np.uint32))
