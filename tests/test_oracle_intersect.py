"""Pins of the oracle's intersection: the watertight ray/triangle test
(Woop, Benthin, Wald, JCGT 2013) on textbook cases, watertightness of
closed meshes, and bit-exact agreement of the oracle's own BVH with brute
force (closest hit by (t, id) order, so the answer is traversal-independent).
"""
import numpy as np
import pytest

import oracle
from paper_2605_27323_amd import scenes


def test_axis_aligned_exact_t():
    v0, v1, v2 = (-1, -1, 5), (1, -1, 5), (0, 1, 5)
    hit, t, b1, b2 = oracle.tri_test((0, 0, 0), (0, 0, 1), v0, v1, v2)
    assert hit and t == 5.0
    # barycentric reconstruction of the hit point (0,0,5)
    p = np.array(v0) + b1 * (np.array(v1) - v0) + b2 * (np.array(v2) - v0)
    assert np.allclose(p, (0, 0, 5), atol=1e-6)
    # back side: double sided
    hit, t, _, _ = oracle.tri_test((0, 0, 10), (0, 0, -1), v0, v1, v2)
    assert hit and t == 5.0
    # behind the origin and parallel rays miss
    assert not oracle.tri_test((0, 0, 6), (0, 0, 1), v0, v1, v2)[0]
    assert not oracle.tri_test((0, 0, 0), (1, 0, 0), v0, v1, v2)[0]
    # other axes, exact distances
    hit, t, _, _ = oracle.tri_test((3, 0.1, 0.1), (-1, 0, 0), (0, -1, -1), (0, 1, -1), (0, 0, 1))
    assert hit and t == 3.0
    hit, t, _, _ = oracle.tri_test((0.25, -2, 0.25), (0, 1, 0), (-1, 0.5, -1), (1, 0.5, -1), (0, 0.5, 1))
    assert hit and t == 2.5


def test_edges_and_vertices_inclusive():
    v0, v1, v2 = (0, 0, 1), (1, 0, 1), (0, 1, 1)
    # exactly on a vertex, on an edge midpoint, on the hypotenuse
    for target in [(0, 0), (1, 0), (0, 1), (0.5, 0), (0, 0.5), (0.5, 0.5)]:
        hit, t, _, _ = oracle.tri_test((target[0], target[1], 0), (0, 0, 1), v0, v1, v2)
        assert hit and t == 1.0, target
    # just outside
    hit = oracle.tri_test((0.5, -1e-6, 0), (0, 0, 1), v0, v1, v2)[0]
    assert not hit


def test_shared_edge_no_gap_no_escape():
    # a quad split on its diagonal: rays exactly on the diagonal hit at least one
    p, i = scenes.quad((-1, -1, 2), (1, -1, 2), (1, 1, 2), (-1, 1, 2))
    tris = p[i]
    rng = np.random.default_rng(0)
    for s in rng.uniform(-1, 1, 200):
        o = (float(s), float(s), 0.0)  # on the diagonal x == y
        d = (0.0, 0.0, 1.0)
        hits = [oracle.tri_test(o, d, *tris[k])[0] for k in range(2)]
        assert any(hits)


def _closed_mesh_scene(pos, idx):
    nt = idx.shape[0]
    return {"positions": pos.astype(np.float32), "indices": idx.astype(np.int32),
            "tri_mat": np.zeros(nt, np.int32), "materials": np.array([[0, 1, 1.5, 0]], np.float32),
            "albedo": np.full((nt, 3), 0.5, np.float32), "emission": np.zeros((nt, 3), np.float32),
            "sky": np.zeros(3, np.float32)}


@pytest.mark.parametrize("kind", ["ico", "box"])
def test_watertight_rays_from_inside_never_escape(kind):
    if kind == "ico":
        up, ui = scenes.icosphere_unit(3)
        pos = 0.7 * up + np.array([0.1, -0.2, 0.3])
        idx = ui
        centre = np.array([0.1, -0.2, 0.3])
    else:
        pos, idx = scenes.box_mesh((-0.5, -0.25, -1.0), (0.75, 0.5, 0.25), 3)
        centre = np.array([0.125, 0.125, -0.375])
    S = oracle.Scene(_closed_mesh_scene(pos, idx), bvh=False)
    p32 = pos.astype(np.float32)
    tris = p32[idx]
    targets = [p32, (tris[:, 0] + tris[:, 1]) / 2, (tris[:, 1] + tris[:, 2]) / 2, (tris[:, 0] + tris[:, 2]) / 2]
    targets = np.concatenate(targets).astype(np.float32)
    rng = np.random.default_rng(1)
    origins = np.concatenate([np.repeat(centre[None], len(targets), 0),
                              centre + rng.uniform(-0.1, 0.1, size=(len(targets), 3))]).astype(np.float32)
    tt = np.concatenate([targets, targets])
    d = tt - origins
    t, prim, _, _ = S.closest(origins, d, mode=0)
    assert (prim >= 0).all(), f"{(prim < 0).sum()} rays escaped"


def _bvh_vs_brute(scene, n_rays, seed):
    Sb = oracle.Scene(scene, bvh=True)
    rng = np.random.default_rng(seed)
    pos = scene["positions"]
    idx = scene["indices"]
    tris = pos[idx]
    lo, hi = pos.min(0) - 0.5, pos.max(0) + 0.5
    o = rng.uniform(lo, hi, size=(n_rays, 3)).astype(np.float32)
    # half of the rays aimed at vertices / edge midpoints / centroids
    k = n_rays // 2
    ti = rng.integers(0, len(idx), k)
    choice = rng.integers(0, 5, k)
    tgt = np.where(choice[:, None] == 0, tris[ti, 0],
          np.where(choice[:, None] == 1, (tris[ti, 0] + tris[ti, 1]) / 2,
          np.where(choice[:, None] == 2, (tris[ti, 1] + tris[ti, 2]) / 2,
          np.where(choice[:, None] == 3, tris[ti, 2], tris[ti].mean(1)))))
    d = rng.normal(size=(n_rays, 3)).astype(np.float32)
    d[:k] = (tgt - o[:k]).astype(np.float32)
    # some axis-parallel rays and origins on coarse grid planes
    ax = rng.integers(0, 3, n_rays // 8)
    d[-len(ax):] = 0
    d[-len(ax):][np.arange(len(ax)), ax] = rng.choice([-1.0, 1.0], len(ax))
    o[-len(ax) // 2:] = np.round(o[-len(ax) // 2:] * 4) / 4
    tb, pb, b1b, b2b = Sb.closest(o, d, mode=0)
    tv, pv, b1v, b2v = Sb.closest(o, d, mode=1)
    assert np.array_equal(pb, pv)
    assert np.array_equal(tb.view(np.uint32), tv.view(np.uint32))
    assert np.array_equal(b1b.view(np.uint32), b1v.view(np.uint32))
    occ_b = Sb.anyhit(o, d, 1.0, mode=0)
    occ_v = Sb.anyhit(o, d, 1.0, mode=1)
    assert np.array_equal(occ_b, occ_v)
    return (pb >= 0).mean()


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_bvh_equals_brute_force_random_soup(seed):
    scene = scenes.random_soup(seed, 64)
    frac = _bvh_vs_brute(scene, 4000, seed)
    assert frac > 0.3


def test_bvh_equals_brute_force_structured():
    scene, _ = scenes.cornell()
    _bvh_vs_brute(scene, 4000, 11)
    scene, _ = scenes.procedural(seed=9, n_objects=6, width=8, height=8)
    _bvh_vs_brute(scene, 3000, 12)


def test_bvh_equals_brute_force_coplanar_duplicates():
    # duplicated coplanar triangles: ties broken by the smaller id on both paths
    p, i = scenes.quad((-1, 0, -1), (-1, 0, 1), (1, 0, 1), (1, 0, -1))
    pos = np.concatenate([p, p, p + [0, 0.25, 0]])
    idx = np.concatenate([i, i + 4, i + 8])
    scene = _closed_mesh_scene(pos, idx)
    _bvh_vs_brute(scene, 2000, 13)
    S = oracle.Scene(scene)
    t, prim, _, _ = S.closest(np.array([[0.1, 2, 0.2]], np.float32), np.array([[0, -1, 0]], np.float32))
    assert t[0] == 1.75 and prim[0] in (4, 5)
