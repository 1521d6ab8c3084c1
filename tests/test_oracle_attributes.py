"""Pins of the oracle's shading attributes and coated material.

The paper's shading stage rebuilds the hit's vertex attributes (normals,
texture coordinates) from the triangle and its barycentrics (Sec. 2.3) and
evaluates a layered material (Sec. 3, OpenPBR).  The oracle's synthetic
subset is checked against what geometry and optics fix:

* shading normals: the vertex normal at each vertex; turned to the
  geometric side; zero or absent -> geometric normal; on a finely
  tessellated sphere with radial vertex normals they approximate the true
  sphere normal to second order in the edge length (a swapped barycentric
  or vertex fails that); in a two-level scene they map by the inverse
  transpose of the instance's map (checked against the flattened scene with
  normals mapped in binary64);
* a plane whose shading normals are all tilted by a under a uniform sky
  L: the fraction of the cosine lobe about the shading normal that lies
  above the geometric plane is (1 + cos a) / 2, so a Lambertian plane of
  albedo r returns r L (1 + cos a) / 2 (rays below the plane are dropped);
* coated material: black base and a smooth coat reflect exactly the
  Fresnel fraction F(cos t) of a uniform sky; with a white base the sky
  seen through the coat adds (1 - F(cos t)) r (1 - Fbar) with Fbar the
  cosine-weighted hemispherical mean of F (fp64 quadrature of the textbook
  Fresnel equations); at ior 1 the material is Lambertian; f is symmetric;
  sampling matches its pdf (chi-square) and its weights f cos / pdf; the
  directional albedo stays <= 1;
* checker texture: each sample on a cell interior equals albedo * t * L
  exactly, t in {1, 1/4} by the parity of floor(u f) + floor(v f) computed
  with integers;
* light sampling on and off agree (paired, 4 sigma) in a room with a
  smooth-shaded coated sphere, a coated box and a textured floor.
"""
import numpy as np
import pytest

import oracle
from paper_2605_27323_amd import scenes

LAMBERT, COATED = scenes.LAMBERT, scenes.COATED


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def fresnel(ci, eta):
    """Unpolarised Fresnel reflectance of a dielectric interface (Born and
    Wolf), ci the cosine on the incident side, eta = n_t / n_i."""
    ci = np.asarray(ci, np.float64)
    st2 = (1.0 - ci * ci) / eta ** 2
    ct = np.sqrt(np.maximum(1.0 - st2, 0.0))
    rs = (ci - eta * ct) / (ci + eta * ct)
    rp = (eta * ci - ct) / (eta * ci + ct)
    return np.where(st2 >= 1.0, 1.0, 0.5 * (rs * rs + rp * rp))


def fresnel_hemi_mean(eta, n=200000):
    mu = (np.arange(n) + 0.5) / n
    return float(2.0 * (fresnel(mu, eta) * mu).sum() / n)


def one_triangle(normals=None, uvs=None, mat=(LAMBERT, 1.0, 1.5, 0.0)):
    pos = np.array([[0, 0, 0], [1, 0, 0], [0, 0, -1]], np.float32)  # normal +y
    sc = {"positions": pos, "indices": np.array([[0, 1, 2]], np.int32), "tri_mat": np.zeros(1, np.int32),
          "materials": np.array([mat], np.float32), "albedo": np.full((1, 3), 0.5, np.float32),
          "emission": np.zeros((1, 3), np.float32), "sky": np.ones(3, np.float32)}
    if normals is not None:
        sc["normals"] = np.asarray(normals, np.float32)
    if uvs is not None:
        sc["uvs"] = np.asarray(uvs, np.float32)
    return sc


# ---------------------------------------------------------------------------
# shading normals
# ---------------------------------------------------------------------------
def test_shading_normal_equals_vertex_normal_at_vertices():
    rng = np.random.default_rng(1)
    for _ in range(50):
        n = rng.normal(size=(3, 3)) * rng.uniform(0.1, 10, size=(3, 1))
        n[:, 1] = np.abs(n[:, 1]) + 0.05  # on the geometric (+y) side
        S = oracle.Scene(one_triangle(normals=n))
        for k, (b1, b2) in enumerate([(0.0, 0.0), (1.0, 0.0), (0.0, 1.0)]):
            ns = S.shading_normal(0, b1, b2)
            assert np.allclose(ns, _unit(n[k]), atol=3e-7), (k, ns, _unit(n[k]))
        # the midpoint of the edge v1 v2: the normalised mean of n1 and n2
        ns = S.shading_normal(0, 0.5, 0.5)
        assert np.allclose(ns, _unit(n[1] + n[2]), atol=3e-7)


def test_shading_normal_turned_to_geometric_side_and_fallbacks():
    n = np.array([[0.3, -1.0, 0.2]] * 3)
    S = oracle.Scene(one_triangle(normals=n))
    assert np.allclose(S.shading_normal(0, 0.2, 0.3), -_unit(n[0]), atol=3e-7)
    ng = np.array([0.0, 1.0, 0.0])
    assert np.allclose(oracle.Scene(one_triangle(normals=np.zeros((3, 3)))).shading_normal(0, 0.2, 0.3), ng)
    assert np.allclose(oracle.Scene(one_triangle()).shading_normal(0, 0.2, 0.3), ng)
    # opposite vertex normals cancel at the midpoint: geometric normal
    n2 = np.array([[1.0, 0.5, 0.0], [-1.0, -0.5, 0.0], [0.0, 0.0, 0.0]])
    assert np.allclose(oracle.Scene(one_triangle(normals=n2)).shading_normal(0, 0.5, 0.0), ng)
    with pytest.raises(ValueError):
        oracle.Scene(one_triangle(normals=np.array([[np.nan, 1, 0]] * 3)))


def _sphere_scene(level, smooth):
    up, ui = scenes.icosphere_unit(level)
    sc = {"positions": up.astype(np.float32), "indices": ui, "tri_mat": np.zeros(len(ui), np.int32),
          "materials": np.array([[LAMBERT, 1.0, 1.5, 0.0]], np.float32),
          "albedo": np.full((len(ui), 3), 0.5, np.float32), "emission": np.zeros((len(ui), 3), np.float32),
          "sky": np.ones(3, np.float32)}
    if smooth:
        sc["normals"] = up.astype(np.float32)
    return sc


def _sphere_rays(n, seed):
    rng = np.random.default_rng(seed)
    o = _unit(rng.normal(size=(n, 3))) * 3.0
    tgt = rng.uniform(-0.5, 0.5, size=(n, 3))
    return o.astype(np.float32), _unit(tgt - o).astype(np.float32)


def test_smooth_sphere_normals_approximate_the_sphere():
    o, d = _sphere_rays(3000, 2)
    err = {}
    for smooth in (False, True):
        S = oracle.Scene(_sphere_scene(4, smooth))
        t, prim, b1, b2 = S.closest(o, d)
        assert (prim >= 0).all()
        x = o.astype(np.float64) + t[:, None] * d
        ns = np.array([S.shading_normal(p, u, v) for p, u, v in zip(prim, b1, b2)])
        err[smooth] = np.degrees(np.arccos(np.clip((ns * _unit(x)).sum(1), -1, 1)))
    # edge of a level-4 icosphere ~ 3.7 degrees: flat facets err by up to
    # about half of it, interpolated normals by a small fraction
    assert err[False].max() > 1.0
    assert err[True].max() < 0.25, err[True].max()
    assert err[True].mean() < 0.1 * err[False].mean()


def test_instanced_normals_map_by_inverse_transpose():
    sc = _sphere_scene(3, True)
    rng = np.random.default_rng(5)
    Q = scenes.random_rotation(rng)
    Ms = []
    for scale in ([1.0, 1.0, 1.0], [3.0, 0.5, 1.5], [0.4, 2.5, 1.0]):
        A = Q @ np.diag(scale) @ scenes.random_rotation(rng)
        T = rng.uniform(-2, 2, 3)
        Ms.append((A, T))
    nt = sc["indices"].shape[0]
    inst = {"mesh_first": np.array([0], np.int32), "mesh_count": np.array([nt], np.int32),
            "inst_mesh": np.zeros(1, np.int32)}
    for A, T in Ms:
        o2w = np.concatenate([A, T[:, None]], 1)
        Ai = np.linalg.inv(A)
        w2o = np.concatenate([Ai, (-Ai @ T)[:, None]], 1)
        inst_q = dict(inst, o2w=o2w.astype(np.float32).reshape(1, 12), w2o=w2o.astype(np.float32).reshape(1, 12))
        S = oracle.Scene(sc, instances=inst_q)
        flat = scenes.flatten_instances(sc, inst_q)
        # flattened normals: n_w = A^-T n per corner, in binary64
        corner_n = sc["normals"][sc["indices"].reshape(-1)].astype(np.float64)
        flat["normals"] = (corner_n @ np.linalg.inv(A.astype(np.float32).astype(np.float64))).astype(np.float32)
        F = oracle.Scene(flat)
        o, d = _sphere_rays(400, 7)
        o = (o.astype(np.float64) * 3 + T).astype(np.float32)
        d = _unit(T + rng.uniform(-0.3, 0.3, (400, 3)) - o).astype(np.float32)
        t, prim, b1, b2, qi = S.closest(o, d, with_inst=True)
        tf, pf, c1, c2 = F.closest(o, d)
        m = (prim >= 0) & (pf >= 0)
        assert m.sum() > 100
        assert (pf[m] == prim[m]).all()
        for i in np.nonzero(m)[0][:150]:
            a = S.shading_normal(prim[i], b1[i], b2[i], inst=qi[i]).astype(np.float64)
            b = F.shading_normal(pf[i], c1[i], c2[i]).astype(np.float64)
            assert np.linalg.norm(a - b) < 2e-5, (a, b)


# ---------------------------------------------------------------------------
# path loop with shading normals: tilted plane under a sky
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("alpha", [0.0, 30.0, 60.0, 80.0])
def test_tilted_shading_normals_closed_form(alpha):
    a, L = 0.6, 1.0
    scene, cam = scenes.tilted_normal_plane(alpha_deg=alpha, albedo=a, sky=L)
    S = oracle.Scene(scene)
    _, _, ps = S.render(cam, spp=512, max_depth=3, seed=4, nee=True, per_sample=True)
    x = ps[..., 0].astype(np.float64).ravel()
    af = float(np.float32(a))
    # every sample is a L (escaped) or 0 (dropped below the plane)
    assert np.isin(x, [0.0, af * L]).all()
    p = (1 + np.cos(np.radians(alpha))) / 2
    sig = af * L * np.sqrt(max(p * (1 - p), 1e-12) / x.size)
    assert abs(x.mean() - af * L * p) < 4 * sig + 1e-9, (x.mean(), af * L * p, sig)


# ---------------------------------------------------------------------------
# coated material
# ---------------------------------------------------------------------------
def _pixel_cosines(cam):
    """cos of the angle between the plane normal +y and the reversed camera
    ray through each pixel centre."""
    c = oracle.camera(cam).astype(np.float64)
    W, H = cam["width"], cam["height"]
    px, py = np.arange(W * H) % W, np.arange(W * H) // W
    sx = (px + 0.5) / W * 2 - 1
    sy = 1 - (py + 0.5) / H * 2
    d = _unit(sx[:, None] * c[3:6] + sy[:, None] * c[6:9] + c[9:12])
    return -d[:, 1]


@pytest.mark.parametrize("ior,theta", [(1.5, 0.0), (1.5, 60.0), (1.33, 75.0), (2.0, 40.0)])
def test_smooth_coat_black_base_reflects_fresnel(ior, theta):
    scene, cam = scenes.coated_plane(ior=ior, rough=0.0, base=0.0, theta_deg=max(theta, 1e-3))
    if theta == 0.0:
        cam = dict(cam, eye=(0.0, 10.0, 0.0), up=(0.0, 0.0, 1.0))
    S = oracle.Scene(scene)
    _, _, ps = S.render(cam, spp=1024, max_depth=2, seed=8, per_sample=True)
    x = ps[..., 0].astype(np.float64)
    mu = _pixel_cosines(cam)
    F = fresnel(mu, ior)
    exp = F.mean()
    sig = np.sqrt((F * (1 - F)).mean() / x.size)
    assert abs(x.mean() - exp) < 4 * sig + 1e-3 * exp, (x.mean(), exp, sig)


@pytest.mark.parametrize("ior,theta,rho", [(1.5, 20.0, 0.8), (1.5, 60.0, 1.0), (1.8, 45.0, 0.5)])
def test_smooth_coat_white_base_closed_form(ior, theta, rho):
    scene, cam = scenes.coated_plane(ior=ior, rough=0.0, base=rho, theta_deg=theta)
    S = oracle.Scene(scene)
    _, _, ps = S.render(cam, spp=1024, max_depth=2, seed=9, per_sample=True)
    x = ps[..., 0].astype(np.float64)
    mu = _pixel_cosines(cam)
    F = fresnel(mu, ior)
    Fbar = fresnel_hemi_mean(ior)
    rf = float(np.float32(rho))
    exp = (F + (1 - F) * rf * (1 - Fbar)).mean()
    se = x.std() / np.sqrt(x.size)
    assert abs(x.mean() - exp) < 4 * se + 1e-3 * exp, (x.mean(), exp, se)


def _rand_dirs(rng, n):
    v = _unit(rng.normal(size=(n, 3)))
    v[:, 2] = np.abs(v[:, 2]) + 1e-3
    return _unit(v).astype(np.float32)


Z = np.array([0, 0, 1], np.float32)


@pytest.mark.parametrize("rough,ior", [(0.2, 1.5), (0.6, 1.3), (1.0, 2.0)])
def test_coat_reciprocity_and_sample_eval_consistency(rough, ior):
    rng = np.random.default_rng(11)
    alb = np.array([0.9, 0.5, 0.1], np.float32)
    wos, wis = _rand_dirs(rng, 200), _rand_dirs(rng, 200)
    for wo, wi in zip(wos, wis):
        f1, _ = oracle.bsdf_eval(COATED, rough, alb, Z, wo, wi, ior=ior, tex=0.25)
        f2, _ = oracle.bsdf_eval(COATED, rough, alb, Z, wi, wo, ior=ior, tex=0.25)
        assert np.allclose(f1, f2, rtol=2e-5, atol=1e-12), (f1, f2)
    nok = 0
    for wo in wos[:100]:
        ok, wi, wgt, p = oracle.bsdf_sample(COATED, rough, ior, alb, Z, wo, rng.uniform(), rng.uniform(),
                                            rng.uniform(), tex=0.25)
        if not ok:
            continue
        nok += 1
        f, pe = oracle.bsdf_eval(COATED, rough, alb, Z, wo, wi, ior=ior, tex=0.25)
        assert abs(p - pe) <= 1e-6 * pe
        assert np.allclose(wgt, f * wi[2] / pe, rtol=1e-5)
    assert nok > 90


def test_coat_at_index_one_is_lambertian():
    rng = np.random.default_rng(12)
    alb = np.array([0.7, 0.3, 0.2], np.float32)
    for wo, wi in zip(_rand_dirs(rng, 100), _rand_dirs(rng, 100)):
        f, p = oracle.bsdf_eval(COATED, 0.4, alb, Z, wo, wi, ior=1.0)
        assert np.allclose(f, alb / np.pi, rtol=1e-5)
        assert abs(p - wi[2] / np.pi) <= 1e-5 * p
        ok, wj, w, _ = oracle.bsdf_sample(COATED, 0.4, 1.0, alb, Z, wo, rng.uniform(0.01, 1), rng.uniform(),
                                          rng.uniform())
        assert ok and np.allclose(w, alb, rtol=1e-5)


@pytest.mark.parametrize("rough,ior", [(0.05, 1.5), (0.3, 1.5), (0.6, 1.5), (1.0, 1.5), (1.0, 2.2)])
def test_coat_sampling_chi2_and_energy(rough, ior):
    """Chi-square where the midpoint quadrature of the pdf resolves the
    specular lobe (roughness >= 0.3); the energy bound at every roughness."""
    rng = np.random.default_rng(13)
    ones = np.ones(3, np.float32)
    for cos_o in (0.95, 0.5, 0.15):
        wo = np.array([np.sqrt(1 - cos_o ** 2), 0.0, cos_o], np.float32)
        N = 20000
        nt, nph = 8, 8
        counts = np.zeros((nt, nph))
        wsum = 0.0
        w2 = 0.0
        u = rng.uniform(size=(N, 3))
        for k in range(N):
            ok, wi, w, _ = oracle.bsdf_sample(COATED, rough, ior, ones, Z, wo, *u[k])
            if not ok:
                continue
            wsum += float(w[0])
            w2 += float(w[0]) ** 2
            th = np.arccos(np.clip(wi[2], -1, 1))
            ph = np.arctan2(wi[1], wi[0]) % (2 * np.pi)
            counts[min(int(th / (np.pi / 2) * nt), nt - 1), min(int(ph / (2 * np.pi) * nph), nph - 1)] += 1
        # directional albedo at a white base: at most 1 (energy)
        mean = wsum / N
        se = np.sqrt(max(w2 / N - mean ** 2, 0) / N)
        assert mean < 1.0 + 4 * se, (cos_o, mean, se)
        assert mean > 0.5
        if rough < 0.3:
            continue
        sub = 10 if cos_o > 0.3 else 40  # the grazing lobe is narrow in phi
        exp = np.zeros((nt, nph))
        for i in range(nt):
            th = (i + (np.arange(sub) + 0.5) / sub) * (np.pi / 2) / nt
            for j in range(nph):
                ph = (j + (np.arange(sub) + 0.5) / sub) * 2 * np.pi / nph
                acc = 0.0
                for t_ in th:
                    for p_ in ph:
                        d = np.array([np.sin(t_) * np.cos(p_), np.sin(t_) * np.sin(p_), np.cos(t_)], np.float32)
                        acc += oracle.bsdf_eval(COATED, rough, ones, Z, wo, d, ior=ior)[1] * np.sin(t_)
                exp[i, j] = N * acc * (np.pi / 2 / nt / sub) * (2 * np.pi / nph / sub)
        m = exp > 20
        chi2 = ((counts[m] - exp[m]) ** 2 / exp[m]).sum()
        dof = m.sum()
        assert chi2 < dof + 6 * np.sqrt(2 * dof) + 0.01 * N, (cos_o, chi2, dof)


# ---------------------------------------------------------------------------
# checker texture
# ---------------------------------------------------------------------------
def test_texture_parity_matches_integer_floor():
    rng = np.random.default_rng(14)
    for _ in range(300):
        uv = rng.uniform(-20, 20, size=(3, 2)).astype(np.float32)
        freq = float(np.float32(rng.choice([0.5, 1.0, 3.0, 7.25])))
        S = oracle.Scene(one_triangle(uvs=uv))
        u, v = uv[0]
        cu = int(np.floor(np.float64(np.float32(u * np.float32(freq)))))
        cv = int(np.floor(np.float64(np.float32(v * np.float32(freq)))))
        exp = 0.25 if (cu + cv) % 2 else 1.0
        assert S.texture(0, 0.0, 0.0, freq) == exp
    assert oracle.Scene(one_triangle(uvs=np.full((3, 2), 0.5))).texture(0, 0.3, 0.3, 0.0) == 1.0
    assert oracle.Scene(one_triangle()).texture(0, 0.3, 0.3, 4.0) == 1.0


def test_checker_plane_samples_are_exact():
    freq, a, L = 4.0, 0.8, 1.0
    scene, cam = scenes.checker_plane(freq=freq, albedo=a, sky=L)
    S = oracle.Scene(scene)
    _, _, ps = S.render(cam, spp=16, max_depth=2, seed=3, per_sample=True)
    W, H = cam["width"], cam["height"]
    c = oracle.camera(cam).astype(np.float64)
    af = np.float32(a)
    checked = {0.25: 0, 1.0: 0}
    for pix in range(W * H):
        px, py = pix % W, pix // W
        corners = []
        for dx in (0.0, 1.0):
            for dy in (0.0, 1.0):
                sx = (px + dx) / W * 2 - 1
                sy = 1 - (py + dy) / H * 2
                d = sx * c[3:6] + sy * c[6:9] + c[9:12]
                t = -c[1] / d[1]
                corners.append(c[:3] + t * d)
        corners = np.array(corners)
        if np.abs(corners[:, [0, 2]]).max() > 0.999:
            continue
        cu = np.floor((corners[:, 0] + 0.13) * freq)
        cv = np.floor((corners[:, 2] + 0.37) * freq)
        # the footprint (plus a margin of rounding) inside one cell only
        mu = np.floor((corners[:, 0] + 0.13) * freq + np.array([[-1e-4], [1e-4]]))
        mv = np.floor((corners[:, 2] + 0.37) * freq + np.array([[-1e-4], [1e-4]]))
        if len(set(cu)) > 1 or len(set(cv)) > 1 or len(set(mu.ravel())) > 1 or len(set(mv.ravel())) > 1:
            continue
        t = 0.25 if (int(cu[0]) + int(cv[0])) % 2 else 1.0
        exp = np.float32(af * np.float32(t)) * np.float32(L)
        assert (ps[pix] == exp).all(), (pix, ps[pix], exp)
        checked[t] += 1
    assert checked[0.25] > 50 and checked[1.0] > 50, checked


# ---------------------------------------------------------------------------
# light sampling on / off with attributes and coats
# ---------------------------------------------------------------------------
def test_nee_on_off_agree_with_attributes():
    scene, cam = scenes.cornell_attributes(coat=(0.25, 1.5))
    cam = dict(cam, width=32, height=32)
    S = oracle.Scene(scene)
    kw = dict(spp=256, max_depth=5, seed=21, per_sample=True)
    _, _, on = S.render(cam, nee=True, **kw)
    _, _, off = S.render(cam, nee=False, **kw)
    d = (on.astype(np.float64) - off).reshape(-1, 3)
    se = d.std(0) / np.sqrt(d.shape[0])
    assert (np.abs(d.mean(0)) < 4 * se).all(), (d.mean(0), se)
    # on the pixels that see the smooth coated sphere
    c = oracle.camera(cam).astype(np.float64)
    px, py = np.arange(1024) % 32, np.arange(1024) // 32
    sx = (px + 0.5) / 32 * 2 - 1
    sy = 1 - (py + 0.5) / 32 * 2
    dirs = _unit(sx[:, None] * c[3:6] + sy[:, None] * c[6:9] + c[9:12]).astype(np.float32)
    o = np.repeat(c[None, :3], 1024, 0).astype(np.float32)
    _, prim, _, _ = S.closest(o, dirs)
    sphere = (prim >= 10) & (prim < 10 + 320)
    assert sphere.sum() > 40
    dd = (on.astype(np.float64) - off)[sphere].reshape(-1, 3)
    se = dd.std(0) / np.sqrt(dd.shape[0])
    assert (np.abs(dd.mean(0)) < 4 * se).all(), (dd.mean(0), se)


@pytest.mark.parametrize("alpha", [40.0, 70.0])
def test_nee_on_off_agree_on_tilted_plane_under_light(alpha):
    """Strongly tilted shading normals under a quad light: light sampling
    must weigh by the same shading cosine and geometric-side rule as BSDF
    sampling."""
    scene, cam = scenes.plane_under_light(albedo=0.7, le=4.0, light_half=0.8, light_h=1.0, half=4.0,
                                          width=16, height=16)
    al = np.radians(alpha)
    nrm = np.zeros((scene["positions"].shape[0], 3), np.float32)
    nrm[:4] = [np.sin(al), np.cos(al), 0.0]
    scene["normals"] = nrm
    S = oracle.Scene(scene)
    kw = dict(spp=512, max_depth=1, seed=31, per_sample=True)
    _, _, on = S.render(cam, nee=True, **kw)
    _, _, off = S.render(cam, nee=False, **kw)
    d = (on.astype(np.float64) - off).reshape(-1, 3)
    se = d.std(0) / np.sqrt(d.shape[0])
    assert (np.abs(d.mean(0)) < 4 * se).all(), (d.mean(0), se)
    assert on.mean() > 0.05


def test_light_behind_the_surface_does_not_leak():
    """A light under a plane with tilted shading normals: directions toward
    it lie on the shading side but below the geometric surface; neither
    light sampling nor BSDF sampling may reach it (only the light above
    counts), so both estimators agree and the image matches that of the
    scene without the light below in expectation."""
    a = 0.7
    P0, I0 = scenes.quad((-4, 0, -4), (-4, 0, 4), (4, 0, 4), (4, 0, -4))
    P1, I1 = scenes.quad((-0.8, 1, -0.8), (0.8, 1, -0.8), (0.8, 1, 0.8), (-0.8, 1, 0.8))    # faces -y
    P2, I2 = scenes.quad((-3, -0.5, -3), (-3, -0.5, 3), (3, -0.5, 3), (3, -0.5, -3))        # faces +y
    al = np.radians(60.0)

    def build(with_below):
        P = [P0, P1] + ([P2] if with_below else [])
        I = [I0, I1 + 4] + ([I2 + 8] if with_below else [])
        nt = 2 * len(P)
        sc = {"positions": np.concatenate(P).astype(np.float32), "indices": np.concatenate(I).astype(np.int32),
              "tri_mat": np.zeros(nt, np.int32), "materials": np.array([[LAMBERT, 1.0, 1.5, 0.0]], np.float32),
              "albedo": np.array([[a] * 3] * 2 + [[0.0] * 3] * (nt - 2), np.float32),
              "emission": np.array([[0.0] * 3] * 2 + [[4.0] * 3] * (nt - 2), np.float32),
              "sky": np.zeros(3, np.float32)}
        nrm = np.zeros((4 * len(P), 3), np.float32)
        nrm[:4] = [np.sin(al), np.cos(al), 0.0]
        sc["normals"] = nrm
        return sc

    cam = dict(eye=(0.0, 0.5, -3.0), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), vfov_deg=45.0, width=16,
               height=16)
    kw = dict(spp=256, max_depth=1, seed=32, per_sample=True)
    S = oracle.Scene(build(True))
    _, _, on = S.render(cam, nee=True, **kw)
    _, _, off = S.render(cam, nee=False, **kw)
    d = (on.astype(np.float64) - off).reshape(-1, 3)
    se = d.std(0) / np.sqrt(d.shape[0])
    assert (np.abs(d.mean(0)) < 4 * se).all(), (d.mean(0), se)
    _, _, ref = oracle.Scene(build(False)).render(cam, nee=True, **kw)
    x, y = on.astype(np.float64).reshape(-1, 3), ref.astype(np.float64).reshape(-1, 3)
    se = np.sqrt(x.var(0) / len(x) + y.var(0) / len(y))
    assert (np.abs(x.mean(0) - y.mean(0)) < 4 * se).all(), (x.mean(0), y.mean(0), se)
    assert y.mean() > 0.02
