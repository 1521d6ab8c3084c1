"""Pins of the oracle's gradient (binary64, stored path with suffix sums).

With sampling independent of albedo and emission (cosine/VNDF sampling,
area-proportional light picks, no roulette) the fixed-sample estimator is a
polynomial in the albedos and linear in the emissions, so:
* the white-furnace gradient has a closed form,
* an emission perturbation changes the image exactly linearly,
* central differences of the binary32 forward agree with it closely.
"""
import numpy as np
import pytest

import oracle
from paper_2605_27323_amd import scenes


@pytest.mark.parametrize("a,D", [(0.5, 3), (0.3, 6), (0.9, 1)])
def test_furnace_gradient_closed_form(a, D):
    le = 1.25
    scene, cam = scenes.furnace(albedo=a, le=le, n=1, width=6, height=5)
    S = oracle.Scene(scene)
    npix = 30
    dimg = np.ones((npix, 3), np.float32)
    ga, ge, aa, ae = S.backward(cam, dimg, spp=3, max_depth=D, seed=2, nee=False)
    af = float(np.float32(a))
    # sum over triangles of dI/d albedo = Le * sum_k k a^(k-1), per pixel
    exp_a = npix * le * sum(k * af ** (k - 1) for k in range(1, D + 1))
    exp_e = npix * sum(af ** k for k in range(D + 1))
    assert np.allclose(ga.sum(0), exp_a, rtol=1e-12)
    assert np.allclose(ge.sum(0), exp_e, rtol=1e-12)
    assert (aa >= np.abs(ga) - 1e-15).all() and (ae >= np.abs(ge) - 1e-15).all()


def loss_of(S, cam, dimg, **kw):
    img, _ = S.render(cam, **kw)
    return float((img.astype(np.float64) * dimg).sum())


def _scene_with_conductor():
    scene, cam = scenes.cornell()
    scene = {k: v.copy() for k, v in scene.items()}
    mats = np.array([[0, 1.0, 1.5, 0], [1, 0.35, 1.5, 0]], np.float32)
    scene["materials"] = mats
    tm = scene["tri_mat"].copy()
    tm[10:22] = 1  # tall box: rough conductor
    scene["tri_mat"] = tm
    return scene, dict(cam, width=20, height=20)


@pytest.mark.parametrize("which", ["lambert", "conductor", "attributes"])
def test_gradient_vs_central_differences(which):
    """attributes: smooth-shaded coated sphere, coated box, checker-textured
    floor (the coat's lobe choice depends on Fresnel only, not on the
    albedo, so the estimator stays a polynomial in the albedos)."""
    scene, cam = scenes.cornell()
    cam = dict(cam, width=20, height=20)
    if which == "conductor":
        scene, cam = _scene_with_conductor()
    if which == "attributes":
        scene, cam = scenes.cornell_attributes(coat=(0.3, 1.5))
        cam = dict(cam, width=20, height=20)
    S = oracle.Scene(scene)
    rng = np.random.default_rng(3)
    npix = cam["width"] * cam["height"]
    dimg = rng.normal(size=(npix, 3)).astype(np.float32)
    kw = dict(spp=2, max_depth=3, seed=4, nee=True)
    ga, ge, _, _ = S.backward(cam, dimg, **kw)
    alb0 = scene["albedo"].copy()
    emi0 = scene["emission"].copy()
    h = 1e-2
    checked = 0
    # albedo: the triangles with the largest gradients (the two largest of
    # each material), all channels
    mag = np.abs(ga).sum(1)
    cand = []
    for m in np.unique(scene["tri_mat"]):
        idx = np.nonzero(scene["tri_mat"] == m)[0]
        cand += list(idx[np.argsort(-mag[idx])[:2]])
    mats_checked = set()
    for t in sorted(set(cand) | set(np.argsort(-mag)[:6])):
        for c in range(3):
            if abs(ga[t, c]) < 1e-3:
                continue
            ap = alb0.copy(); ap[t, c] += h
            am = alb0.copy(); am[t, c] -= h
            S.set_params(ap, emi0); lp = loss_of(S, cam, dimg, **kw)
            S.set_params(am, emi0); lm = loss_of(S, cam, dimg, **kw)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - ga[t, c]) <= 1e-2 * abs(ga[t, c]), (t, c, fd, ga[t, c])
            checked += 1
            mats_checked.add(int(scene["tri_mat"][t]))
    S.set_params(alb0, emi0)
    assert checked >= 6
    assert mats_checked == set(np.unique(scene["tri_mat"]).tolist()), mats_checked
    # emission of the light (linear: any step is exact up to binary32 rounding)
    for t in np.nonzero(emi0.any(1))[0]:
        for c in range(3):
            ep = emi0.copy(); ep[t, c] += 1.0
            S.set_params(alb0, ep); lp = loss_of(S, cam, dimg, **kw)
            S.set_params(alb0, emi0); l0 = loss_of(S, cam, dimg, **kw)
            assert abs((lp - l0) - ge[t, c]) <= 1e-3 * abs(ge[t, c]) + 1e-5, (t, c, lp - l0, ge[t, c])
    # a non-emitting triangle gains emission gradient from direct hits
    assert np.abs(ge[:10]).sum() > 0


def test_gradient_linear_in_dimage():
    scene, cam = scenes.cornell()
    cam = dict(cam, width=12, height=12)
    S = oracle.Scene(scene)
    rng = np.random.default_rng(5)
    d1 = rng.normal(size=(144, 3)).astype(np.float32)
    d2 = rng.normal(size=(144, 3)).astype(np.float32)
    kw = dict(spp=2, max_depth=4, seed=6)
    g1 = S.backward(cam, d1, **kw)
    g2 = S.backward(cam, d2, **kw)
    g12 = S.backward(cam, (d1.astype(np.float64) + d2).astype(np.float32), **kw)
    for k in range(2):
        ref = g1[k] + g2[k]
        # d1 + d2 is rounded to binary32: bound by the absolute terms
        bound = 1e-6 * (g1[k + 2] + g2[k + 2]) + 1e-12
        assert (np.abs(g12[k] - ref) <= bound).all()
