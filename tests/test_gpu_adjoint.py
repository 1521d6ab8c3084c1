"""GPU path-replay adjoint (through the C ABI and the autograd function)
against the oracle's binary64 stored-path gradient and against central
finite differences of the GPU forward.

Tolerances: per entry |g - g*| <= 1e-4 * (sum of absolute terms) +
1e-7 * max|g*| (fp32 atomic sums of signed terms make a plain relative error
of a near-zero sum meaningless), and ||g - g*|| / ||g*|| <= 1e-4 globally;
central differences with h = 1e-3: relative 1e-2.
"""
import numpy as np
import pytest

import oracle
from paper_2605_27323_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2605_27323_amd import ptmi  # noqa: E402


def log(*a):
    print(*a, flush=True)


def _grad_check(ga, ge, oa, oe, aa, ae):
    for g, o, a in [(ga, oa, aa), (ge, oe, ae)]:
        err = np.abs(g.astype(np.float64) - o)
        bound = 1e-4 * a + 1e-7 * np.abs(o).max()
        assert (err <= bound).all(), (err.max(), int((err > bound).sum()))
        assert np.linalg.norm(g - o) <= 1e-4 * np.linalg.norm(o)


def _conductor_cornell():
    scene, cam = scenes.cornell()
    scene = {k: v.copy() for k, v in scene.items()}
    scene["materials"] = np.array([[0, 1.0, 1.5, 0], [1, 0.35, 1.5, 0]], np.float32)
    scene["tri_mat"][10:22] = 1
    return scene, cam


@pytest.mark.parametrize("which", ["cornell", "conductor", "procedural"])
def test_adjoint_vs_oracle(which):
    if which == "cornell":
        scene, cam = scenes.cornell()
        cam = dict(cam, width=64, height=48)
    elif which == "conductor":
        scene, cam = _conductor_cornell()
        cam = dict(cam, width=64, height=48)
    else:
        scene, cam = scenes.procedural(seed=61, n_objects=30, width=80, height=50)
    log("adjoint vs oracle", which)
    R = ptmi.Renderer(scene, cam)
    rng = np.random.default_rng(1)
    n = cam["width"] * cam["height"]
    d = rng.normal(size=(n, 3)).astype(np.float32)
    kw = dict(spp=3, max_depth=5, seed=7, frame=1)
    ga = torch.zeros_like(R.albedo)
    ge = torch.zeros_like(R.emission)
    R.backward(torch.from_numpy(d).cuda(), ga, ge, **kw)
    ga, ge = ga.cpu().numpy()[:R.nt], ge.cpu().numpy()[:R.nt]
    oa, oe, aa, ae = oracle.Scene(scene).backward(cam, d, **kw)
    _grad_check(ga, ge, oa, oe, aa, ae)


def test_adjoint_accumulates_and_rejects_roulette():
    scene, cam = scenes.cornell()
    cam = dict(cam, width=16, height=16)
    R = ptmi.Renderer(scene, cam)
    d = torch.ones((16, 16, 3), dtype=torch.float32, device="cuda")
    g1a, g1e = torch.zeros_like(R.albedo), torch.zeros_like(R.emission)
    R.backward(d, g1a, g1e, spp=1, max_depth=3)
    g2a, g2e = g1a.clone(), g1e.clone()
    R.backward(d, g2a, g2e, spp=1, max_depth=3)
    assert torch.allclose(g2a, 2 * g1a, rtol=1e-5, atol=1e-6)
    with pytest.raises(ptmi.PtError):
        R.backward(d, g1a, g1e, spp=1, max_depth=3, rr_start=2)


def test_adjoint_vs_central_differences_and_autograd():
    scene, cam = _conductor_cornell()
    cam = dict(cam, width=48, height=40)
    log("finite differences")
    R = ptmi.Renderer(scene, cam)
    rng = np.random.default_rng(2)
    target = torch.from_numpy(rng.uniform(0, 1, size=(40, 48, 3)).astype(np.float32)).cuda()
    kw = dict(spp=4, max_depth=4, seed=5, mode="wave")
    alb = R.albedo.clone().requires_grad_(True)
    emi = R.emission.clone().requires_grad_(True)
    img = ptmi.render_differentiable(alb, emi, R, **kw)
    loss = ((img - target) ** 2).sum()
    loss.backward()
    ga, ge = alb.grad.cpu().numpy(), emi.grad.cpu().numpy()

    def loss_at(a, e):
        R.albedo.copy_(torch.from_numpy(a).cuda())
        R.emission.copy_(torch.from_numpy(e).cuda())
        I = R.render(**kw).double()
        return float(((I - target.double()) ** 2).sum())

    a0 = alb.detach().cpu().numpy()
    e0 = emi.detach().cpu().numpy()
    h = 1e-3
    checked = 0
    order = np.argsort(-np.abs(ga).sum(1))
    for t in order[:16]:
        for c in range(3):
            if abs(ga[t, c]) < 1e-2 or a0[t, c] < 2 * h:
                continue
            ap = a0.copy(); ap[t, c] += h
            am = a0.copy(); am[t, c] -= h
            fd = (loss_at(ap, e0) - loss_at(am, e0)) / (2 * h)
            assert abs(fd - ga[t, c]) <= 1e-2 * abs(ga[t, c]) + 1e-3, (t, c, fd, ga[t, c])
            checked += 1
    for t in [34, 35]:
        for c in range(3):
            ep = e0.copy(); ep[t, c] += h
            em = e0.copy(); em[t, c] -= h
            fd = (loss_at(a0, ep) - loss_at(a0, em)) / (2 * h)
            assert abs(fd - ge[t, c]) <= 1e-2 * abs(ge[t, c]) + 1e-3, (t, c, fd, ge[t, c])
            checked += 1
    assert checked >= 20


def _primary_counts(scene, cam, spp):
    """Primary-hit samples per triangle (pixel-centre rays, times spp), from
    the oracle's closest hit."""
    c = oracle.camera(cam)
    W, H = cam["width"], cam["height"]
    px, py = np.meshgrid(np.arange(W), np.arange(H))
    sx = ((px + 0.5) / W * 2 - 1).astype(np.float32).reshape(-1, 1)
    sy = (1 - (py + 0.5) / H * 2).astype(np.float32).reshape(-1, 1)
    d = sx * c[3:6] + sy * c[6:9] + c[9:12]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.repeat(c[None, :3], len(d), 0)
    _, prim, _, _ = oracle.Scene(scene).closest(o, d.astype(np.float32))
    return np.bincount(prim[prim >= 0], minlength=scene["indices"].shape[0]) * spp


def test_adam_recovers_perturbed_albedo():
    # reduced differentiable-rendering protocol: target rendered with
    # perturbed per-triangle albedos, 200 Adam steps on the L2 image loss;
    # recovery measured on triangles with >= 64 primary-hit samples.  The
    # loss gradient 2 (I - T) dI/dalbedo is estimated with independent
    # samples for I and for the adjoint (the same samples would bias it by
    # Var(I) / albedo).
    scene, cam = scenes.cornell()
    cam = dict(cam, width=64, height=64)
    R = ptmi.Renderer(scene, cam)
    true_alb = scenes.perturb_albedo(scene["albedo"], seed=5, sigma=0.05)
    true_alb[34:] = 0.0  # the light keeps albedo 0
    kw = dict(spp=4, max_depth=4)
    R.albedo.copy_(torch.from_numpy(true_alb).cuda())
    target = R.render(seed=999, spp=256, max_depth=4).clone()
    alb = torch.from_numpy(scene["albedo"].copy()).cuda().requires_grad_(True)
    opt = torch.optim.Adam([alb], lr=5e-3)
    for step in range(200):
        opt.zero_grad()
        R.albedo.copy_(alb.detach())
        I = R.render(seed=2 * step, **kw)
        d_img = (2.0 / I.numel()) * (I - target)
        ga = torch.zeros_like(R.albedo)
        ge = torch.zeros_like(R.emission)
        R.backward(d_img.contiguous(), ga, ge, seed=2 * step + 1, **kw)
        alb.grad = ga
        opt.step()
        with torch.no_grad():
            alb.clamp_(0.02, 0.95)
            alb[34:] = 0.0
    seen = np.nonzero(_primary_counts(scene, cam, kw["spp"]) >= 64)[0]
    seen = seen[seen < 34]
    a_true = true_alb[seen]
    e0 = float(np.abs(scene["albedo"][seen] - a_true).mean())
    e1 = float(np.abs(alb.detach().cpu().numpy()[seen] - a_true).mean())
    log("albedo error over", len(seen), "triangles:", e0, "->", e1)
    assert len(seen) >= 12
    assert e1 < 0.5 * e0


def test_adjoint_halton_sampler_vs_oracle():
    scene, cam = scenes.procedural(seed=62, n_objects=25, width=64, height=40)
    log("adjoint halton")
    R = ptmi.Renderer(scene, cam)
    d = np.random.default_rng(2).normal(size=(64 * 40, 3)).astype(np.float32)
    kw = dict(spp=3, max_depth=5, seed=4, frame=2)
    ga = torch.zeros_like(R.albedo)
    ge = torch.zeros_like(R.emission)
    R.backward(torch.from_numpy(d).cuda(), ga, ge, sampler="halton", **kw)
    ga, ge = ga.cpu().numpy()[:R.nt], ge.cpu().numpy()[:R.nt]
    oa, oe, aa, ae = oracle.Scene(scene).backward(cam, d, sampler=1, **kw)
    _grad_check(ga, ge, oa, oe, aa, ae)


@pytest.mark.parametrize("mode", ["mega", "wave", "mega_keep_hits", "wave_keep_hits"])
def test_adjoint_replay_schedules_match_oracle(mode):
    # replay A as the megakernel-style kernel or as the wavefront stages
    # (with the hybrid tail), or keeping its intersections for replay B:
    # the same per-path radiance and the same terms, so all gradients match
    # the oracle's to the atomics' rounding
    scene, cam = scenes.procedural(seed=62, n_objects=30, width=72, height=48)
    log("adjoint replay", mode)
    R = ptmi.Renderer(scene, cam)
    rng = np.random.default_rng(4)
    n = cam["width"] * cam["height"]
    d = rng.normal(size=(n, 3)).astype(np.float32)
    kw = dict(spp=3, max_depth=5, seed=9, frame=2)
    extra = {"wave": dict(mode="wave", tail_threshold=500, tail_bounce=3), "mega": dict(mode="mega"),
             "mega_keep_hits": dict(mode="mega", flags=ptmi.FLAG_KEEP_HITS),
             "wave_keep_hits": dict(mode="wave", tail_threshold=500, tail_bounce=3, flags=ptmi.FLAG_KEEP_HITS)}[mode]
    ga = torch.zeros_like(R.albedo)
    ge = torch.zeros_like(R.emission)
    R.backward(torch.from_numpy(d).cuda(), ga, ge, **kw, **extra)
    st = R.stats()
    # replay B traces the forward frame's rays again: the counts are those
    # of the forward megakernel with the same arguments
    R.render(mode="mega", **kw)
    fst = R.stats()
    assert st["extension_rays"] == fst["extension_rays"] > 0
    assert st["shadow_rays"] == fst["shadow_rays"] > 0
    ga, ge = ga.cpu().numpy()[:R.nt], ge.cpu().numpy()[:R.nt]
    oa, oe, aa, ae = oracle.Scene(scene).backward(cam, d, **kw)
    _grad_check(ga, ge, oa, oe, aa, ae)


def test_adjoint_keep_hits_full_size_matches_tracing_replay():
    # the benchmark's backward (1.02M triangles, 512x512, 8 spp, depth 6)
    # with replay B reading replay A's records against replay B tracing
    # again: the same terms, summed by atomics in another order
    scene, _ = scenes.procedural(seed=2, n_objects=2000)
    cam = dict(eye=(0.0, 50.0, -130.0), target=(0.0, 40.0, 0.0), up=(0.0, 1.0, 0.0), vfov_deg=50.0,
               width=512, height=512)
    R = ptmi.Renderer(scene, cam)
    log("adjoint keep hits full size", R.nt)
    d = torch.ones((512, 512, 3), dtype=torch.float32, device="cuda")
    kw = dict(spp=8, max_depth=6, seed=0, frame=3, block=256, grid_mult=8, stack_lds=8)
    out = []
    # the tracing replay, then the kept records written by the megakernel-
    # style replay A and by the wavefront stages with the hybrid tail
    for flags, extra in ((0, dict(mode="mega")), (ptmi.FLAG_KEEP_HITS, dict(mode="mega")),
                         (ptmi.FLAG_KEEP_HITS, dict(mode="wave", tail_threshold=1 << 18, tail_bounce=4))):
        ga = torch.zeros_like(R.albedo)
        ge = torch.zeros_like(R.emission)
        R.backward(d, ga, ge, flags=flags, **kw, **extra)
        st = R.stats()
        out.append((ga.cpu().numpy()[:R.nt].astype(np.float64), ge.cpu().numpy()[:R.nt].astype(np.float64),
                    st["extension_rays"], st["shadow_rays"]))
    a0, e0, n0, s0 = out[0]
    assert n0 > 0 and s0 > 0
    for a1, e1, n1, s1 in out[1:]:
        assert n1 == n0 and s1 == s0
        for g0, g1 in ((a0, a1), (e0, e1)):
            assert np.abs(g0).sum() > 0
            assert np.linalg.norm(g1 - g0) <= 1e-5 * np.linalg.norm(g0)
