"""Pins of the oracle's materials, light and camera sampling against closed
forms, quadrature and sampling statistics (binary64 checks of the
binary32 oracle functions)."""
import numpy as np
import pytest

import oracle
from paper_2605_27323_amd import scenes

LAMBERT, CONDUCTOR, DIELECTRIC = 0, 1, 2


def sphere_grid(n_theta=96, n_phi=192):
    """Midpoint quadrature over the upper hemisphere: directions, weights."""
    th = (np.arange(n_theta) + 0.5) * (np.pi / 2) / n_theta
    ph = (np.arange(n_phi) + 0.5) * 2 * np.pi / n_phi
    T, P = np.meshgrid(th, ph, indexing="ij")
    dirs = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    w = (np.sin(T) * (np.pi / 2 / n_theta) * (2 * np.pi / n_phi)).reshape(-1)
    return dirs, w


def test_lambert_eval_sample_exact():
    alb = np.array([0.63, 0.06, 0.05], np.float32)
    n = np.array([0, 0, 1], np.float32)
    wo = np.array([0.3, -0.2, 0.9], np.float32)
    wo /= np.linalg.norm(wo)
    f, pdf = oracle.bsdf_eval(LAMBERT, 1.0, alb, n, wo, np.array([0.0, 0.6, 0.8], np.float32))
    assert np.array_equal(f, alb * np.float32(1.0 / np.pi))
    assert abs(pdf - 0.8 / np.pi) < 1e-7
    rng = np.random.default_rng(0)
    for _ in range(200):
        u = rng.uniform(0, 1, 3).astype(np.float32)
        ok, wi, w, p = oracle.bsdf_sample(LAMBERT, 1.0, 1.5, alb, n, wo, *u)
        assert ok and np.array_equal(w, alb) and wi[2] > 0
        assert abs(np.linalg.norm(wi) - 1) < 1e-6
        assert abs(p - wi[2] / np.pi) < 1e-6


def test_lambert_sampling_chi2_cosine():
    n = np.array([0.0, 0.0, 1.0], np.float32)
    wo = np.array([0.0, 0.0, 1.0], np.float32)
    rng = np.random.default_rng(1)
    N = 20000
    cos2 = np.empty(N)
    for i in range(N):
        ok, wi, w, p = oracle.bsdf_sample(LAMBERT, 1.0, 1.5, np.ones(3, np.float32), n, wo, 0.5,
                                          rng.uniform(), rng.uniform())
        cos2[i] = wi[2] ** 2
    # cosine-weighted: cos^2(theta) is uniform on [0,1]
    h = np.bincount(np.minimum((cos2 * 32).astype(int), 31), minlength=32)
    chi2 = ((h - N / 32) ** 2 / (N / 32)).sum()
    assert chi2 < 31 + 6 * np.sqrt(62)


@pytest.mark.parametrize("rough", [0.3, 0.5, 0.8])
def test_conductor_reciprocity_energy_and_pdf(rough):
    alb = np.array([1.0, 1.0, 1.0], np.float32)
    n = np.array([0, 0, 1], np.float32)
    dirs, w = sphere_grid(64, 128)
    rng = np.random.default_rng(2)
    for ct in [0.95, 0.6, 0.2]:
        st = np.sqrt(1 - ct * ct)
        wo = np.array([st, 0, ct], np.float32)
        fs = np.zeros(len(dirs))
        ps = np.zeros(len(dirs))
        for i, d in enumerate(dirs.astype(np.float32)):
            f, p = oracle.bsdf_eval(CONDUCTOR, rough, alb, n, wo, d)
            fs[i] = f[0]
            ps[i] = p
        albedo_integral = (fs * dirs[:, 2] * w).sum()
        pdf_integral = (ps * w).sum()
        assert albedo_integral <= 1.0 + 2e-2, albedo_integral
        assert pdf_integral <= 1.0 + 2e-2, pdf_integral
        if rough <= 0.3 and ct > 0.5:
            assert albedo_integral > 0.9
            assert pdf_integral > 0.9
        # reciprocity
        for _ in range(20):
            a = rng.normal(size=3)
            a[2] = abs(a[2])
            a = (a / np.linalg.norm(a)).astype(np.float32)
            f1, _ = oracle.bsdf_eval(CONDUCTOR, rough, alb * 0.5, n, wo, a)
            f2, _ = oracle.bsdf_eval(CONDUCTOR, rough, alb * 0.5, n, a, wo)
            assert np.allclose(f1, f2, rtol=1e-4, atol=0)


@pytest.mark.parametrize("rough", [0.05, 0.2])
def test_conductor_energy_by_sampling(rough):
    # E[weight] = integral of f cos over the hemisphere (albedo 1): at most 1,
    # close to 1 for a smooth conductor seen near normal incidence
    n = np.array([0, 0, 1], np.float32)
    wo = np.array([0.3, 0.0, np.sqrt(1 - 0.09)], np.float32)
    rng = np.random.default_rng(8)
    ws = []
    for _ in range(4000):
        ok, wi, wgt, p = oracle.bsdf_sample(CONDUCTOR, rough, 1.5, np.ones(3, np.float32), n, wo, 0.5,
                                            rng.uniform(), rng.uniform())
        ws.append(wgt[0] if ok else 0.0)
    ws = np.array(ws)
    m, se = ws.mean(), ws.std() / np.sqrt(len(ws))
    assert m <= 1.0 + 4 * se + 1e-6
    assert m > 0.95


@pytest.mark.parametrize("rough,tol", [(0.05, 2e-3), (0.1, 2e-3), (0.5, 2e-3)])
def test_conductor_sample_matches_eval(rough, tol):
    # binary32 rounding of the half vector moves a very narrow lobe's D by a
    # relative amount that grows like 1/alpha^2, hence the looser tolerance
    alb = np.array([0.9, 0.5, 0.2], np.float32)
    n = np.array([0, 0, 1], np.float32)
    rng = np.random.default_rng(3)
    wo = np.array([0.5, 0.1, 0.86], np.float32)
    wo /= np.linalg.norm(wo)
    nok = 0
    for _ in range(300):
        ok, wi, wgt, p = oracle.bsdf_sample(CONDUCTOR, rough, 1.5, alb, n, wo, 0.5, rng.uniform(), rng.uniform())
        if not ok:
            continue
        nok += 1
        f, pe = oracle.bsdf_eval(CONDUCTOR, rough, alb, n, wo, wi)
        assert abs(p - pe) <= tol * pe
        assert np.allclose(wgt, f * wi[2] / pe, rtol=1.5 * tol)
    assert nok > 200


def test_conductor_sampling_chi2():
    # sampled directions vs the eval pdf integrated over (theta, phi) cells
    rough = 0.4
    n = np.array([0, 0, 1], np.float32)
    wo = np.array([0.4, 0.0, np.sqrt(1 - 0.16)], np.float32)
    rng = np.random.default_rng(4)
    N = 20000
    nt, nph = 8, 8
    counts = np.zeros((nt, nph))
    for _ in range(N):
        ok, wi, _, _ = oracle.bsdf_sample(CONDUCTOR, rough, 1.5, np.ones(3, np.float32), n, wo, 0.5,
                                          rng.uniform(), rng.uniform())
        if not ok:
            continue
        th = np.arccos(np.clip(wi[2], -1, 1))
        ph = np.arctan2(wi[1], wi[0]) % (2 * np.pi)
        counts[min(int(th / (np.pi / 2) * nt), nt - 1), min(int(ph / (2 * np.pi) * nph), nph - 1)] += 1
    # expected: N * integral of pdf over each cell (sub-sampled midpoint rule)
    sub = 12
    exp = np.zeros((nt, nph))
    for i in range(nt):
        for j in range(nph):
            th = (i + (np.arange(sub) + 0.5) / sub) * (np.pi / 2) / nt
            ph = (j + (np.arange(sub) + 0.5) / sub) * 2 * np.pi / nph
            T, P = np.meshgrid(th, ph, indexing="ij")
            acc = 0.0
            for t_, p_ in zip(T.ravel(), P.ravel()):
                d = np.array([np.sin(t_) * np.cos(p_), np.sin(t_) * np.sin(p_), np.cos(t_)], np.float32)
                acc += oracle.bsdf_eval(CONDUCTOR, rough, np.ones(3, np.float32), n, wo, d)[1] * np.sin(t_)
            exp[i, j] = N * acc * (np.pi / 2 / nt / sub) * (2 * np.pi / nph / sub)
    m = exp > 20
    chi2 = ((counts[m] - exp[m]) ** 2 / exp[m]).sum()
    dof = m.sum()
    assert chi2 < dof + 6 * np.sqrt(2 * dof) + 0.01 * N, (chi2, dof)


def test_dielectric_fresnel_normal_incidence_and_snell():
    ior = 1.5
    n = np.array([0, 0, 1], np.float32)
    wo = np.array([0, 0, 1], np.float32)
    rough = 0.01  # alpha = 1e-4: microfacet normal within ~1e-4 of n
    F0 = ((ior - 1) / (ior + 1)) ** 2
    # the lobe switches from reflection to refraction at u4 = F
    refl = lambda u4: oracle.bsdf_sample(DIELECTRIC, rough, ior, np.ones(3, np.float32), n, wo, u4, 0.3, 0.7)[1][2] > 0
    lo, hi = 0.0, 0.5
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        if refl(mid):
            lo = mid
        else:
            hi = mid
    assert abs(lo - F0) < 1e-5
    # Snell: sin_t = sin_i / ior (entering), with an oblique incidence
    for ci in [0.9, 0.5, 0.2]:
        si = np.sqrt(1 - ci * ci)
        wo = np.array([si, 0, ci], np.float32)
        ok, wi, w, _ = oracle.bsdf_sample(DIELECTRIC, rough, ior, np.ones(3, np.float32), n, wo, 0.999, 0.3, 0.7)
        assert ok and wi[2] < 0
        st = np.sqrt(wi[0] ** 2 + wi[1] ** 2)
        assert abs(st - si / ior) < 2e-3
        assert abs(w[0] - 1 / ior ** 2) < 2e-2 * (1 / ior ** 2)
    # total internal reflection from inside beyond the critical angle
    wo_in = np.array([0.9, 0, -np.sqrt(1 - 0.81)], np.float32)
    for u4 in [0.0, 0.5, 0.999]:
        ok, wi, w, _ = oracle.bsdf_sample(DIELECTRIC, rough, ior, np.ones(3, np.float32), n, wo_in, u4, 0.3, 0.7)
        assert ok and wi[2] < 0  # stays inside (the -n side)


def test_triangle_point_uniform():
    v0, v1, v2 = np.array([0, 0, 0.]), np.array([2, 0, 0.]), np.array([0.5, 1.5, 0.])
    rng = np.random.default_rng(5)
    N = 20000
    pts = np.array([oracle.sample_triangle(v0, v1, v2, rng.uniform(), rng.uniform()) for _ in range(N)])
    # barycentric (b1, b2) from the point, then uniform density => b1 + b2 ~ triangle law
    M = np.stack([v1 - v0, v2 - v0], 1)[:2]
    b = np.linalg.solve(M, (pts[:, :2] - v0[:2]).T).T
    assert (b >= -1e-6).all() and (b.sum(1) <= 1 + 1e-6).all()
    # 16 sub-triangles of equal area: counts uniform
    k = 4
    i = np.minimum((b[:, 0] * k).astype(int), k - 1)
    j = np.minimum((b[:, 1] * k).astype(int), k - 1)
    up = (b[:, 0] * k - i) + (b[:, 1] * k - j) > 1
    cell = (i * k + j) * 2 + up
    valid = i + j < k
    h = np.bincount(cell[valid], minlength=2 * k * k)
    h = h[h > 0]
    assert len(h) == k * k
    e = N / (k * k)
    chi2 = ((h - e) ** 2 / e).sum()
    assert chi2 < 15 + 6 * np.sqrt(30)


def test_light_pick_area_proportional():
    # three emitters with areas 1, 2, 5 (plus a non-emitter)
    pos = np.array([[0, 0, 0], [1, 0, 0], [0, 2, 0], [0, 0, 1], [2, 0, 1], [0, 2, 1],
                    [0, 0, 2], [2, 0, 2], [0, 2, 2], [0, 0, 3], [5, 0, 3], [0, 2, 3]], np.float32)
    idx = np.arange(12, dtype=np.int32).reshape(4, 3)
    emi = np.array([[1, 1, 1], [0, 0, 0], [1, 0, 0], [0, 0, 2]], np.float32)
    scene = {"positions": pos, "indices": idx, "tri_mat": np.zeros(4, np.int32),
             "materials": np.array([[0, 1, 1.5, 0]], np.float32), "albedo": np.full((4, 3), .5, np.float32),
             "emission": emi, "sky": np.zeros(3, np.float32)}
    S = oracle.Scene(scene, bvh=False)
    assert S.num_lights == 3  # triangle 1 is not a light
    # CDF boundaries at 1/8 and 3/8 of 2^32 (areas 1, 2, 5)
    b1, b2 = int(2**32 / 8), int(3 * 2**32 / 8)
    assert S.pick_light(0) == 0 and S.pick_light(b1) == 0 and S.pick_light(b1 + 1) == 1
    assert S.pick_light(b2) == 1 and S.pick_light(b2 + 1) == 2 and S.pick_light(2**32 - 1) == 2
    rng = np.random.default_rng(6)
    picks = np.array([S.pick_light(int(w)) for w in rng.integers(0, 2**32, 20000, dtype=np.uint64)])
    frac = np.bincount(picks, minlength=3) / len(picks)
    assert np.allclose(frac, [1 / 8, 2 / 8, 5 / 8], atol=0.015)


def test_offset_moves_to_normal_side():
    # o = p + 2^-15 m n, m = the triangle's largest coordinate magnitude
    rng = np.random.default_rng(7)
    for _ in range(500):
        tri = rng.uniform(-100, 100, (3, 3)).astype(np.float32) * np.float32(10.0 ** rng.uniform(-3, 1))
        b = rng.dirichlet([1, 1, 1])
        p = (b @ tri.astype(np.float64)).astype(np.float32)
        if rng.uniform() < 0.2:
            p[rng.integers(0, 3)] = np.float32(0.0)
        nvec = rng.normal(size=3)
        nvec = (nvec / np.linalg.norm(nvec)).astype(np.float32)
        q = oracle.offset(p, nvec, tri)
        m = max(float(np.abs(tri).max()), 2.0 ** -7)
        dlt = q.astype(np.float64) - p
        assert np.dot(dlt, nvec) > 0
        # each coordinate moves by 2^-15 m n_c, up to the rounding of the sum
        ulp = np.spacing(np.abs(q).astype(np.float32)).astype(np.float64)
        assert (np.abs(dlt - 2.0 ** -15 * m * nvec) <= ulp + 1e-30).all(), (dlt, m, nvec)


def test_offset_clears_large_triangle_near_coordinate_plane():
    # a ground quad of half-width 1000 at y = 0: the continuation ray leaving
    # a hit near the origin upward never hits the quad again (a step of a
    # fixed size near zero, below the rounding of the 1000-scale vertices,
    # did about 1 time in 8)
    scene, cam = scenes.plane_under_sky(albedo=0.5, sky=1.0, half=1000.0, width=16, height=16)
    cam = dict(cam, vfov_deg=2.0)
    S = oracle.Scene(scene)
    _, _, ps = S.render(cam, spp=256, max_depth=3, seed=1, per_sample=True)
    assert (ps == np.float32(0.5)).all()


def test_camera_centre_and_fov():
    cam = dict(eye=(1.0, 2.0, 3.0), target=(1.0, 2.0, -7.0), up=(0.0, 1.0, 0.0), vfov_deg=60.0, width=4, height=2)
    c = oracle.camera(cam)
    E, R, U, F = c[:3], c[3:6], c[6:9], c[9:]
    assert np.array_equal(E, np.array([1, 2, 3], np.float32))
    assert np.allclose(F, [0, 0, -1]) and np.allclose(U, [0, np.tan(np.pi / 6), 0], rtol=1e-7)
    # right vector scaled by tan(vfov/2) * W/H
    assert np.allclose(R, [2 * np.tan(np.pi / 6), 0, 0], rtol=1e-7)  # F x up = +x
    # the top image edge is vfov/2 above the axis: angle between F and F + U
    top = F + U
    ang = np.degrees(np.arccos(np.dot(top, F) / np.linalg.norm(top)))
    assert abs(ang - 30.0) < 1e-4
