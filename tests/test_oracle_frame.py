"""Pins of the oracle's local shading frame (Duff, Burgess, Christensen,
Hery, Kensler, Liani, Villemin, "Building an Orthonormal Basis, Revisited",
JCGT 2017) and of its materials at normals other than +z.

The frame maps directions between world space and the local space where
the BSDFs are written (normal = +z); the materials' own pins use n = +z, so
these pin the frame: orthonormality and handedness over random normals
(including n.z < 0 and n.z near -1, where the construction switches
branch), and BSDF values, pdfs and sampling at tilted normals against the
same BSDF at +z in a frame the test builds itself in binary64.
"""
import numpy as np
import pytest

import oracle

LAMBERT, CONDUCTOR, DIELECTRIC = 0, 1, 2


def normals(seed=0, n=400):
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    special = [(0, 0, 1), (0, 0, -1), (1, 0, 0), (0, 1, 0), (0, -1, 0), (-1, 0, 0),
               (1e-4, -2e-4, -1), (3e-4, 1e-4, 1), (0.6, 0.0, -0.8), (0.0, -0.6, -0.8),
               (1e-7, 0, -1), (0, 0, -1e-30), (0.7, 0.7, -1e-6)]
    v = np.concatenate([v, np.array(special, np.float64)])
    v[:40, 2] = -np.abs(v[:40, 2]) - 3.0  # a batch with n.z close to -1
    return (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)


def test_frame_orthonormal_right_handed():
    for n in normals():
        t, b = oracle.frame(n)
        t, b, nn = t.astype(np.float64), b.astype(np.float64), n.astype(np.float64)
        for u in (t, b):
            assert abs(np.linalg.norm(u) - 1) < 1e-6, (n, t, b)
            assert abs(np.dot(u, nn)) < 1e-6, (n, t, b)
        assert abs(np.dot(t, b)) < 1e-6, (n, t, b)
        assert np.abs(np.cross(t, b) - nn).max() < 2e-6, (n, t, b)


def own_frame(n):
    """A binary64 orthonormal frame around n built independently (Gram-Schmidt)."""
    n = np.asarray(n, np.float64)
    a = np.array([1.0, 0, 0]) if abs(n[0]) < 0.9 else np.array([0, 1.0, 0])
    t = a - np.dot(a, n) * n
    t /= np.linalg.norm(t)
    return t, np.cross(n, t), n


def to_world(fr, l):
    t, b, n = fr
    return l[0] * t + l[1] * b + l[2] * n


def rand_local(rng, upper=True):
    v = rng.normal(size=3)
    v /= np.linalg.norm(v)
    if upper:
        v[2] = abs(v[2])
    return v


@pytest.mark.parametrize("mtype,rough", [(LAMBERT, 1.0), (CONDUCTOR, 0.3), (CONDUCTOR, 0.7)])
def test_eval_at_tilted_normals_equals_eval_at_z(mtype, rough):
    rng = np.random.default_rng(1)
    alb = np.array([0.9, 0.4, 0.2], np.float32)
    z = np.array([0, 0, 1], np.float32)
    for n in normals(2, 60):
        fr = own_frame(n)
        for _ in range(6):
            lo, li = rand_local(rng), rand_local(rng)
            if lo[2] < 0.05 or li[2] < 0.05:
                continue
            wo, wi = to_world(fr, lo).astype(np.float32), to_world(fr, li).astype(np.float32)
            f1, p1 = oracle.bsdf_eval(mtype, rough, alb, n, wo, wi)
            f0, p0 = oracle.bsdf_eval(mtype, rough, alb, z, lo.astype(np.float32), li.astype(np.float32))
            assert np.allclose(f1, f0, rtol=2e-4, atol=1e-9), (n, lo, li, f1, f0)
            assert abs(p1 - p0) <= 2e-4 * p0 + 1e-9, (n, p1, p0)


@pytest.mark.parametrize("mtype,rough", [(LAMBERT, 1.0), (CONDUCTOR, 0.4)])
def test_sample_at_tilted_normals_matches_eval(mtype, rough):
    rng = np.random.default_rng(3)
    alb = np.array([0.8, 0.5, 0.3], np.float32)
    nok = 0
    for n in normals(4, 80):
        fr = own_frame(n)
        lo = rand_local(rng)
        if lo[2] < 0.1:
            continue
        wo = to_world(fr, lo).astype(np.float32)
        for _ in range(4):
            ok, wi, w, p = oracle.bsdf_sample(mtype, rough, 1.5, alb, n, wo, 0.5, rng.uniform(), rng.uniform())
            if not ok:
                continue
            nok += 1
            assert abs(np.linalg.norm(wi.astype(np.float64)) - 1) < 2e-6
            cos_i = float(np.dot(wi.astype(np.float64), n))
            assert cos_i > 0, (n, wi)
            f, pe = oracle.bsdf_eval(mtype, rough, alb, n, wo, wi)
            assert abs(p - pe) <= 3e-3 * pe, (n, p, pe)
            assert np.allclose(w, f * cos_i / pe, rtol=5e-3), (n, w, f * cos_i / pe)
    assert nok > 250


def test_lambert_sampling_chi2_at_tilted_normal():
    # cosine-weighted about n: cos^2 uniform on [0, 1], azimuth uniform in
    # a frame the test builds itself
    rng = np.random.default_rng(5)
    N = 16000
    for n in normals(6, 3)[:1].tolist() + [[0.0, 0.6, -0.8], [1e-4, 0.0, -1.0]]:
        n = np.asarray(n, np.float32)
        n /= np.linalg.norm(n)
        fr = own_frame(n)
        cos2 = np.empty(N)
        phi = np.empty(N)
        for i in range(N):
            ok, wi, _, _ = oracle.bsdf_sample(LAMBERT, 1.0, 1.5, np.ones(3, np.float32), n, n, 0.5,
                                              rng.uniform(), rng.uniform())
            w = wi.astype(np.float64)
            c = np.dot(w, fr[2])
            cos2[i] = c * c
            phi[i] = np.arctan2(np.dot(w, fr[1]), np.dot(w, fr[0])) % (2 * np.pi)
        for x, k in [(cos2, 32), (phi / (2 * np.pi), 32)]:
            h = np.bincount(np.minimum((x * k).astype(int), k - 1), minlength=k)
            chi2 = ((h - N / k) ** 2 / (N / k)).sum()
            assert chi2 < (k - 1) + 6 * np.sqrt(2 * (k - 1)), (n, chi2)


def test_dielectric_at_tilted_normal_snell_and_reflection():
    # outside normal n tilted; entering from outside and leaving from inside
    ior = 1.5
    rough = 0.01  # alpha = 1e-4
    rng = np.random.default_rng(7)
    for n in normals(8, 40):
        fr = own_frame(n)
        nn = n.astype(np.float64)
        for inside in (False, True):
            lo = rand_local(rng)
            if lo[2] < 0.2:
                continue
            if inside:
                lo[2] = -lo[2]
            wo = to_world(fr, lo).astype(np.float32)
            eta = 1 / ior if inside else ior
            ci = abs(float(np.dot(wo.astype(np.float64), nn)))
            si = np.sqrt(max(0.0, 1 - ci * ci))
            # refraction (u4 close to 1): other side, sin_t = sin_i / eta
            ok, wi, w, _ = oracle.bsdf_sample(DIELECTRIC, rough, ior, np.ones(3, np.float32), n, wo, 0.999999,
                                              0.3, 0.7)
            if si / eta < 0.95:
                assert ok
                wd = wi.astype(np.float64)
                side = np.sign(np.dot(wd, nn))
                assert side == (1.0 if inside else -1.0), (n, inside, wo, wi)
                st = np.linalg.norm(np.cross(wd, nn))
                assert abs(st - si / eta) < 2e-3, (st, si / eta)
                assert abs(w[0] - 1 / eta ** 2) < 2e-2 / eta ** 2, (w, eta)
            # reflection (u4 = 0): same side, mirror direction
            ok, wi, w, _ = oracle.bsdf_sample(DIELECTRIC, rough, ior, np.ones(3, np.float32), n, wo, 0.0, 0.3, 0.7)
            assert ok
            wd = wi.astype(np.float64)
            mirror = 2 * np.dot(wo.astype(np.float64), nn) * nn - wo
            assert np.abs(wd - mirror).max() < 2e-3, (n, inside, wd, mirror)
