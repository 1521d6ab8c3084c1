"""Pins of the oracle's path tracer against closed forms of the light
transport equation (paper Eq. 1) and the unbiasedness of its Monte Carlo
estimator (Eq. 2-3).

* White furnace: inside a closed, inward-facing cube where every triangle has
  albedo a and emits Le, every path with light sampling and roulette off
  collects exactly Le * sum_{k=0..D} a^k (the D-bounce truncation of
  Le / (1 - a)).
* Diffuse plane under a uniform sky: a Lambertian weight equals the albedo
  exactly and one bounce escapes, so a plane pixel is exactly a * L_sky.
* Lambert's polygon formula: radiance off a diffuse plane lit by one quad
  light is (a / pi) E(x), E the polygon irradiance.
"""
import numpy as np
import pytest

import oracle
from paper_2605_27323_amd import scenes


@pytest.mark.parametrize("a", [0.0, 0.3, 0.5, 0.9])
@pytest.mark.parametrize("D", [0, 1, 5, 32])
def test_white_furnace_exact_without_nee(a, D):
    le = 1.5
    scene, cam = scenes.furnace(albedo=a, le=le, n=2, width=8, height=8)
    S = oracle.Scene(scene)
    img, frag, ps = S.render(cam, spp=2, max_depth=D, seed=3, nee=False, per_sample=True)
    af = float(np.float32(a))
    expect = le * sum(af ** k for k in range(D + 1))
    tol = (2 * D + 4) * 2.0 ** -24 * expect + 1e-30
    assert np.abs(ps - expect).max() <= tol, (ps.min(), ps.max(), expect)


@pytest.mark.parametrize("nee,rr", [(True, -1), (True, 2), (False, 1)])
def test_white_furnace_statistical(nee, rr):
    a, le, D = 0.5, 1.0, 6
    scene, cam = scenes.furnace(albedo=a, le=le, n=2, width=16, height=16)
    S = oracle.Scene(scene)
    _, _, ps = S.render(cam, spp=64, max_depth=D, seed=5, nee=nee, rr_start=rr, per_sample=True)
    x = ps[..., 0].ravel().astype(np.float64)
    expect = le * (1 - a ** (D + 1)) / (1 - a)
    se = x.std() / np.sqrt(x.size)
    assert abs(x.mean() - expect) < 4 * se + 1e-7, (x.mean(), expect, se)
    if not nee and rr < 0:
        assert se == 0


@pytest.mark.parametrize("nee", [False, True])
def test_plane_under_sky_exact(nee):
    a, sky = 0.6, 1.25
    scene, cam = scenes.plane_under_sky(albedo=a, sky=sky, width=24, height=20)
    S = oracle.Scene(scene)
    af = float(np.float32(a) * np.float32(sky))
    for D in [1, 3]:
        _, _, ps = S.render(cam, spp=3, max_depth=D, seed=1, nee=nee, per_sample=True)
        vals = set(np.unique(ps).tolist())
        assert vals <= {af, float(np.float32(sky))}, vals
        plane = (ps[..., 0] == np.float32(af)).mean()
        assert 0.2 < plane < 0.8
    _, _, ps0 = S.render(cam, spp=3, max_depth=0, seed=1, nee=nee, per_sample=True)
    assert set(np.unique(ps0).tolist()) <= {0.0, float(np.float32(sky))}
    # D = 0: samples on the plane carry no light; sky samples keep the sky
    assert ((ps0[..., 0] == 0) == (ps[..., 0] == np.float32(af))).all()


def polygon_irradiance(x, n, verts, le):
    """Lambert's formula: E = le/2 * sum_i angle(r_i, r_i+1) * n . unit(r_i x r_i+1)."""
    e = 0.0
    k = len(verts)
    for i in range(k):
        r0 = verts[i] - x
        r1 = verts[(i + 1) % k] - x
        r0 = r0 / np.linalg.norm(r0)
        r1 = r1 / np.linalg.norm(r1)
        c = np.cross(r0, r1)
        ang = np.arccos(np.clip(np.dot(r0, r1), -1, 1))
        e += ang * np.dot(n, c / np.linalg.norm(c))
    return abs(0.5 * le * e)


@pytest.mark.parametrize("nee", [True, False])
def test_lambert_polygon_irradiance(nee):
    a, le = 0.5, 4.0
    scene, _ = scenes.plane_under_light(albedo=a, le=le, width=6, height=6)
    # look straight down through a narrow field of view so that E(x) is close
    # to linear across each pixel's jitter footprint
    cam = dict(eye=(0.8, 0.5, 0.3), target=(0.8, 0.0, 0.3), up=(0.0, 0.0, 1.0), vfov_deg=10.0,
               width=6, height=6)
    S = oracle.Scene(scene)
    spp = 2048 if nee else 8192
    img, _, ps = S.render(cam, spp=spp, max_depth=1, seed=7, nee=nee, per_sample=True)
    # pixel-centre primary hits
    c = oracle.camera(cam)
    E, R, U, F = c[:3].astype(np.float64), c[3:6], c[6:9], c[9:]
    verts = np.array(scene["positions"][4:8], np.float64)
    ok = 0
    for pix in range(36):
        px, py = pix % 6, pix // 6
        sx = (px + 0.5) / 6 * 2 - 1
        sy = 1 - (py + 0.5) / 6 * 2
        d = sx * R + sy * U + F
        d = d / np.linalg.norm(d)
        if d[1] >= 0:
            continue
        t = -E[1] / d[1]
        x = E + t * d
        if abs(x[0]) > 3.5 or abs(x[2]) > 3.5:
            continue
        expect = a / np.pi * polygon_irradiance(x, np.array([0, 1.0, 0]), verts, le)
        s = ps[pix, :, 0].astype(np.float64)
        se = s.std() / np.sqrt(s.size)
        # jitter inside the pixel moves x; E is smooth there, so allow 0.2% on top of 4 sigma
        assert abs(s.mean() - expect) < 4 * se + 0.002 * expect, (pix, s.mean(), expect, se)
        ok += 1
    assert ok == 36


def test_nee_on_off_agree_cornell():
    scene, cam = scenes.cornell()
    cam = dict(cam, width=32, height=32)
    S = oracle.Scene(scene)
    m = []
    for nee in [True, False]:
        _, _, ps = S.render(cam, spp=64, max_depth=5, seed=11, nee=nee, per_sample=True)
        x = ps.reshape(-1, 3).astype(np.float64)
        m.append((x.mean(0), x.std(0) / np.sqrt(x.shape[0])))
    diff = np.abs(m[0][0] - m[1][0])
    se = np.sqrt(m[0][1] ** 2 + m[1][1] ** 2)
    assert (diff < 4 * se).all(), (m, diff, se)
    # light sampling lowers the variance of the direct light
    assert (m[0][1] < m[1][1]).all()


def test_variance_falls_as_one_over_n():
    scene, cam = scenes.cornell()
    cam = dict(cam, width=16, height=16)
    S = oracle.Scene(scene)
    errs = []
    ref, _ = S.render(cam, spp=1024, max_depth=5, seed=100)
    for spp in [4, 64]:
        img, _ = S.render(cam, spp=spp, max_depth=5, seed=1)
        errs.append(((img - ref) ** 2).mean())
    ratio = errs[0] / errs[1]
    assert 8 < ratio < 32, ratio
