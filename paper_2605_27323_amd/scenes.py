"""Seeded synthetic scene and camera generators.

This module only produces input arrays (geometry, per-triangle parameters,
material table, camera).  It holds none of the rendering arithmetic, so both
the HIP renderer and the CPU oracle can be fed from it.

A scene is a dict of NumPy arrays:
    positions  float32 [nv, 3]
    indices    int32   [nt, 3]   counter-clockwise (v0, v1, v2) = front side
    tri_mat    int32   [nt]      index into ``materials``
    materials  float32 [nm, 4]   (type, roughness, ior, 0)
    albedo     float32 [nt, 3]
    emission   float32 [nt, 3]   one-sided, front face only
    sky        float32 [3]       constant radiance of escaped rays
and optionally per-vertex attributes:
    normals    float32 [nv, 3]   shading normals (zero rows: flat shading)
    uvs        float32 [nv, 2]   texture coordinates (for the checker
                                 texture of materials whose 4th entry, the
                                 checker frequency, is > 0)
Material types: LAMBERT, CONDUCTOR, DIELECTRIC, COATED (a GGX dielectric
coat of the material's roughness and ior over a Lambertian base of the
triangle's albedo).
A camera is a dict {eye, target, up, vfov_deg, width, height}.

The paper's own benchmark asset is not available; the procedural scenes
below stand in for it with the sizes and material mix of the workloads
(icospheres and tessellated boxes on a ground plane under quad lights).
"""
from __future__ import annotations

import numpy as np

LAMBERT = 0
CONDUCTOR = 1
DIELECTRIC = 2
COATED = 3


def _pack(pos_list, idx_list, mat_list, alb_list, emi_list, materials, sky=(0.0, 0.0, 0.0)):
    offs = 0
    idx_all = []
    for p, i in zip(pos_list, idx_list):
        idx_all.append(i + offs)
        offs += p.shape[0]
    return {
        "positions": np.ascontiguousarray(np.concatenate(pos_list).astype(np.float32)),
        "indices": np.ascontiguousarray(np.concatenate(idx_all).astype(np.int32)),
        "tri_mat": np.ascontiguousarray(np.concatenate(mat_list).astype(np.int32)),
        "materials": np.ascontiguousarray(np.asarray(materials, dtype=np.float32).reshape(-1, 4)),
        "albedo": np.ascontiguousarray(np.concatenate(alb_list).astype(np.float32)),
        "emission": np.ascontiguousarray(np.concatenate(emi_list).astype(np.float32)),
        "sky": np.asarray(sky, dtype=np.float32),
    }


def quad(p0, p1, p2, p3):
    """Two triangles (p0,p1,p2), (p0,p2,p3); front side given by CCW order."""
    pos = np.array([p0, p1, p2, p3], dtype=np.float64)
    idx = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    return pos, idx


def box_mesh(lo, hi, n=1, outward=True):
    """Axis-aligned box with an n x n grid of quads per face (12 n^2 triangles).

    Vertices live on one (n+1)^3 lattice so that shared edges use the very same
    coordinates (needed for a watertight mesh)."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    g = np.arange(n + 1, dtype=np.float64) / n
    coords = [lo[a] + (hi[a] - lo[a]) * g for a in range(3)]
    for a in range(3):
        coords[a][0], coords[a][-1] = lo[a], hi[a]

    def vid(i, j, k):
        return (i * (n + 1) + j) * (n + 1) + k

    X, Y, Z = np.meshgrid(coords[0], coords[1], coords[2], indexing="ij")
    lattice = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    tris = []
    r = np.arange(n)
    A, B = np.meshgrid(r, r, indexing="ij")
    A = A.ravel()
    B = B.ravel()
    # for each face: fixed axis, fixed side, and the two varying axes (u, v)
    # chosen so that u x v points along the outward normal.
    faces = [
        (0, 0, 2, 1), (0, n, 1, 2),
        (1, 0, 0, 2), (1, n, 2, 0),
        (2, 0, 1, 0), (2, n, 0, 1),
    ]
    for axis, side, ua, va in faces:
        def idx3(a, b):
            ijk = [None, None, None]
            ijk[axis] = np.full_like(a, side)
            ijk[ua] = a
            ijk[va] = b
            return vid(ijk[0], ijk[1], ijk[2])
        q0 = idx3(A, B)
        q1 = idx3(A + 1, B)
        q2 = idx3(A + 1, B + 1)
        q3 = idx3(A, B + 1)
        t1 = np.stack([q0, q1, q2], axis=1)
        t2 = np.stack([q0, q2, q3], axis=1)
        tris.append(np.concatenate([t1, t2]))
    idx = np.concatenate(tris).astype(np.int64)
    # compact the lattice to used vertices
    used, inv = np.unique(idx.ravel(), return_inverse=True)
    pos = lattice[used]
    idx = inv.reshape(-1, 3).astype(np.int32)
    # orient: make every normal point away from the centre (or towards it)
    c = 0.5 * (lo + hi)
    v0, v1, v2 = pos[idx[:, 0]], pos[idx[:, 1]], pos[idx[:, 2]]
    nrm = np.cross(v1 - v0, v2 - v0)
    ctr = (v0 + v1 + v2) / 3.0 - c
    flip = (np.einsum("ij,ij->i", nrm, ctr) < 0) == outward
    idx[flip] = idx[flip][:, [0, 2, 1]]
    return pos, idx


_ICO_CACHE: dict = {}


def icosphere_unit(level):
    """Unit icosphere; level 1 = icosahedron (20 faces), each level x4 faces."""
    if level in _ICO_CACHE:
        return _ICO_CACHE[level]
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    for _ in range(level - 1):
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
        e.sort(axis=1)
        ue, inv = np.unique(e, axis=0, return_inverse=True)
        inv = inv.ravel()
        mid = v[ue[:, 0]] + v[ue[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = v.shape[0]
        v = np.concatenate([v, mid])
        nf = f.shape[0]
        a = base + inv[:nf]
        b = base + inv[nf:2 * nf]
        c = base + inv[2 * nf:]
        f = np.concatenate([
            np.stack([f[:, 0], a, c], 1), np.stack([f[:, 1], b, a], 1),
            np.stack([f[:, 2], c, b], 1), np.stack([a, b, c], 1)])
    # outward orientation check
    v0, v1, v2 = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    n = np.cross(v1 - v0, v2 - v0)
    flip = np.einsum("ij,ij->i", n, v0 + v1 + v2) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    _ICO_CACHE[level] = (v, f.astype(np.int32))
    return _ICO_CACHE[level]


def _tri_params(nt, alb, emi, mat):
    return (np.repeat(np.asarray(mat, np.int32)[None], nt, 0).reshape(nt),
            np.repeat(np.asarray(alb, np.float64)[None], nt, 0),
            np.repeat(np.asarray(emi, np.float64)[None], nt, 0))


# --------------------------------------------------------------------------
# Cornell-style room: 5 walls, two boxes, one quad light (36 triangles)
# --------------------------------------------------------------------------
def cornell(tall_box=None):
    """tall_box: None (white Lambertian) or (roughness, ior) to make the
    tall box a rough dielectric (material 1)."""
    white = (0.73, 0.73, 0.73)
    red = (0.63, 0.06, 0.05)
    green = (0.14, 0.45, 0.09)
    P, I, M, A, E = [], [], [], [], []

    def add(pos, idx, alb, emi=(0, 0, 0), mat=0):
        P.append(pos)
        I.append(idx)
        m, a, e = _tri_params(idx.shape[0], alb, emi, mat)
        M.append(m)
        A.append(a)
        E.append(e)

    # floor y=0 facing +y, ceiling y=2 facing -y, back wall z=-1 facing +z
    add(*quad((-1, 0, -1), (-1, 0, 1), (1, 0, 1), (1, 0, -1)), white)
    add(*quad((-1, 2, -1), (1, 2, -1), (1, 2, 1), (-1, 2, 1)), white)
    add(*quad((-1, 0, -1), (1, 0, -1), (1, 2, -1), (-1, 2, -1)), white)
    # left wall x=-1 facing +x (red), right wall x=+1 facing -x (green)
    add(*quad((-1, 0, -1), (-1, 2, -1), (-1, 2, 1), (-1, 0, 1)), red)
    add(*quad((1, 0, -1), (1, 0, 1), (1, 2, 1), (1, 2, -1)), green)
    add(*box_mesh((-0.7, 0.0, -0.7), (-0.1, 1.2, -0.1), 1), white, mat=0 if tall_box is None else 1)
    add(*box_mesh((0.1, 0.0, -0.2), (0.7, 0.6, 0.4), 1), white)
    # light at y=1.999 facing -y
    add(*quad((-0.25, 1.999, -0.25), (0.25, 1.999, -0.25), (0.25, 1.999, 0.25), (-0.25, 1.999, 0.25)),
        (0.0, 0.0, 0.0), (15.0, 15.0, 15.0))
    mats = [(LAMBERT, 1.0, 1.5, 0.0)]
    if tall_box is not None:
        mats.append((DIELECTRIC, float(tall_box[0]), float(tall_box[1]), 0.0))
    scene = _pack(P, I, M, A, E, mats)
    cam = dict(eye=(0.0, 1.0, 3.6), target=(0.0, 1.0, 0.0), up=(0.0, 1.0, 0.0),
               vfov_deg=40.0, width=128, height=128)
    return scene, cam


def furnace(albedo=0.5, le=1.0, n=2, width=16, height=16):
    """Closed cube [-1,1]^3 with inward-facing triangles, every triangle
    Lambertian with the same albedo and the same inward emission; camera at
    the centre."""
    pos, idx = box_mesh((-1, -1, -1), (1, 1, 1), n, outward=False)
    m, a, e = _tri_params(idx.shape[0], (albedo,) * 3, (le,) * 3, 0)
    scene = _pack([pos], [idx], [m], [a], [e], [(LAMBERT, 1.0, 1.5, 0.0)])
    cam = dict(eye=(0.0, 0.0, 0.0), target=(0.3, 0.2, 1.0), up=(0.0, 1.0, 0.0),
               vfov_deg=90.0, width=width, height=height)
    return scene, cam


def plane_under_sky(albedo=0.6, sky=1.0, half=1.0, width=16, height=16, height_cam=3.0):
    """Two-triangle square at y=0 facing +y under a constant sky; camera above
    looking straight down (the square fills only part of the view)."""
    pos, idx = quad((-half, 0, -half), (-half, 0, half), (half, 0, half), (half, 0, -half))
    m, a, e = _tri_params(2, (albedo,) * 3, (0, 0, 0), 0)
    scene = _pack([pos], [idx], [m], [a], [e], [(LAMBERT, 1.0, 1.5, 0.0)], sky=(sky,) * 3)
    cam = dict(eye=(0.0, height_cam, 0.0), target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0),
               vfov_deg=60.0, width=width, height=height)
    return scene, cam


def slab_over_plane(ior=1.5, rough=0.0, albedo=0.5, sky=1.0, half=1000.0, slab=(1.0, 2.0), width=16,
                    height=16, vfov_deg=2.0):
    """Diffuse square (half-width `half`) at y=0 facing +y under a closed
    dielectric slab (a box spanning the same square, y in `slab`, outward
    normals) and a constant sky; camera at y = 10 looking straight down
    through a narrow field of view."""
    p0, i0 = quad((-half, 0, -half), (-half, 0, half), (half, 0, half), (half, 0, -half))
    p1, i1 = box_mesh((-half, slab[0], -half), (half, slab[1], half), 1)
    m0, a0, e0 = _tri_params(2, (albedo,) * 3, (0, 0, 0), 0)
    m1, a1, e1 = _tri_params(i1.shape[0], (0, 0, 0), (0, 0, 0), 1)
    scene = _pack([p0, p1], [i0, i1], [m0, m1], [a0, a1], [e0, e1],
                  [(LAMBERT, 1.0, 1.5, 0.0), (DIELECTRIC, rough, ior, 0.0)], sky=(sky,) * 3)
    cam = dict(eye=(0.0, 10.0, 0.0), target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0),
               vfov_deg=vfov_deg, width=width, height=height)
    return scene, cam


def emitter_in_slab(ior=1.5, rough=0.0, le=2.0, half=8.0, width=16, height=16):
    """Upward-facing emissive square (y = 1.5, half-width `half`, albedo 0)
    inside a closed dielectric slab (y in [1, 2], same extent, outward
    normals); black sky; camera at y = 10 looking straight down through a
    2-degree field of view."""
    p0, i0 = quad((-half, 1.5, -half), (-half, 1.5, half), (half, 1.5, half), (half, 1.5, -half))
    p1, i1 = box_mesh((-half, 1.0, -half), (half, 2.0, half), 1)
    m0, a0, e0 = _tri_params(2, (0, 0, 0), (le,) * 3, 0)
    m1, a1, e1 = _tri_params(i1.shape[0], (0, 0, 0), (0, 0, 0), 1)
    scene = _pack([p0, p1], [i0, i1], [m0, m1], [a0, a1], [e0, e1],
                  [(LAMBERT, 1.0, 1.5, 0.0), (DIELECTRIC, rough, ior, 0.0)])
    cam = dict(eye=(0.0, 10.0, 0.0), target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0),
               vfov_deg=2.0, width=width, height=height)
    return scene, cam


def tilted_normal_plane(alpha_deg=30.0, albedo=0.6, sky=1.0, half=1000.0, width=8, height=8):
    """Square at y = 0 facing +y whose four vertex normals all equal
    (sin a, cos a, 0): shading normals tilted by a from the geometric
    normal.  Constant sky; camera at y = 10 looking straight down through a
    2-degree field of view."""
    pos, idx = quad((-half, 0, -half), (-half, 0, half), (half, 0, half), (half, 0, -half))
    m, a, e = _tri_params(2, (albedo,) * 3, (0, 0, 0), 0)
    scene = _pack([pos], [idx], [m], [a], [e], [(LAMBERT, 1.0, 1.5, 0.0)], sky=(sky,) * 3)
    al = np.radians(alpha_deg)
    scene["normals"] = np.tile(np.array([np.sin(al), np.cos(al), 0.0], np.float32), (4, 1))
    cam = dict(eye=(0.0, 10.0, 0.0), target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0),
               vfov_deg=2.0, width=width, height=height)
    return scene, cam


def coated_plane(ior=1.5, rough=0.0, base=0.0, sky=1.0, theta_deg=45.0, half=1000.0, width=8, height=8,
                 vfov_deg=0.5):
    """Coated square at y = 0 facing +y (base albedo `base`) under a constant
    sky, seen at `theta_deg` from its normal from 10 units away through a
    narrow field of view."""
    pos, idx = quad((-half, 0, -half), (-half, 0, half), (half, 0, half), (half, 0, -half))
    m, a, e = _tri_params(2, (base,) * 3, (0, 0, 0), 0)
    scene = _pack([pos], [idx], [m], [a], [e], [(COATED, rough, ior, 0.0)], sky=(sky,) * 3)
    th = np.radians(theta_deg)
    cam = dict(eye=(0.0, 10.0 * np.cos(th), -10.0 * np.sin(th)), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0),
               vfov_deg=vfov_deg, width=width, height=height)
    return scene, cam


def checker_plane(freq=4.0, albedo=0.8, sky=1.0, half=1.0, uv_offset=(0.13, 0.37), width=32, height=32):
    """Square at y = 0 facing +y, texture coordinates (x, z) + uv_offset at
    its corners, Lambertian with a checker texture of frequency `freq`;
    constant sky; camera at y = 3 looking straight down (the square fills
    the middle of the view)."""
    pos, idx = quad((-half, 0, -half), (-half, 0, half), (half, 0, half), (half, 0, -half))
    m, a, e = _tri_params(2, (albedo,) * 3, (0, 0, 0), 0)
    scene = _pack([pos], [idx], [m], [a], [e], [(LAMBERT, 1.0, 1.5, float(freq))], sky=(sky,) * 3)
    scene["uvs"] = (pos[:, [0, 2]] + np.asarray(uv_offset)).astype(np.float32)
    cam = dict(eye=(0.0, 3.0, 0.0), target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0),
               vfov_deg=40.0, width=width, height=height)
    return scene, cam


def with_attributes(scene, normals=None, uvs=None):
    """A copy of a scene with vertex attributes added (zero normals and
    zero texture coordinates where not given)."""
    out = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in scene.items()}
    nv = scene["positions"].shape[0]
    out["normals"] = np.zeros((nv, 3), np.float32) if normals is None else np.asarray(normals, np.float32)
    out["uvs"] = np.zeros((nv, 2), np.float32) if uvs is None else np.asarray(uvs, np.float32)
    return out


def cornell_attributes(coat=(0.2, 1.5), freq=6.0):
    """Cornell room with shading attributes: the tall box replaced by a
    smooth-shaded level-3 icosphere with a coat (roughness, ior) over a
    white base, the short box a coated box with flat shading (zero vertex
    normals), a checker-textured floor (texture coordinates (x, z) + 0.1,
    frequency `freq`), the walls flat and untextured."""
    white = (0.73, 0.73, 0.73)
    red = (0.63, 0.06, 0.05)
    green = (0.14, 0.45, 0.09)
    P, I, M, A, E, N, U = [], [], [], [], [], [], []

    def add(pos, idx, alb, emi=(0, 0, 0), mat=0, nrm=None, uv=None):
        P.append(pos)
        I.append(idx)
        m, a, e = _tri_params(idx.shape[0], alb, emi, mat)
        M.append(m); A.append(a); E.append(e)
        N.append(np.zeros((pos.shape[0], 3)) if nrm is None else nrm)
        U.append(np.zeros((pos.shape[0], 2)) if uv is None else uv)

    fp, fi = quad((-1, 0, -1), (-1, 0, 1), (1, 0, 1), (1, 0, -1))
    add(fp, fi, white, mat=2, uv=fp[:, [0, 2]] + 0.1)
    add(*quad((-1, 2, -1), (1, 2, -1), (1, 2, 1), (-1, 2, 1)), white)
    add(*quad((-1, 0, -1), (1, 0, -1), (1, 2, -1), (-1, 2, -1)), white)
    add(*quad((-1, 0, -1), (-1, 2, -1), (-1, 2, 1), (-1, 0, 1)), red)
    add(*quad((1, 0, -1), (1, 0, 1), (1, 2, 1), (1, 2, -1)), green)
    up, ui = icosphere_unit(3)
    add(np.array([-0.4, 0.42, -0.4]) + 0.4 * up, ui, (0.9, 0.9, 0.9), mat=1, nrm=up)
    add(*box_mesh((0.1, 0.0, -0.2), (0.7, 0.6, 0.4), 1), (0.2, 0.4, 0.8), mat=1)
    add(*quad((-0.25, 1.999, -0.25), (0.25, 1.999, -0.25), (0.25, 1.999, 0.25), (-0.25, 1.999, 0.25)),
        (0.0, 0.0, 0.0), (15.0, 15.0, 15.0))
    mats = [(LAMBERT, 1.0, 1.5, 0.0), (COATED, float(coat[0]), float(coat[1]), 0.0),
            (LAMBERT, 1.0, 1.5, float(freq))]
    scene = _pack(P, I, M, A, E, mats)
    scene["normals"] = np.concatenate(N).astype(np.float32)
    scene["uvs"] = np.concatenate(U).astype(np.float32)
    cam = dict(eye=(0.0, 1.0, 3.6), target=(0.0, 1.0, 0.0), up=(0.0, 1.0, 0.0),
               vfov_deg=40.0, width=128, height=128)
    return scene, cam


def plane_under_light(albedo=0.5, le=4.0, light_half=0.5, light_h=1.0, half=4.0,
                      width=16, height=16):
    """Diffuse square at y=0 under one downward-facing quad light (for the
    polygon-irradiance closed form)."""
    p0, i0 = quad((-half, 0, -half), (-half, 0, half), (half, 0, half), (half, 0, -half))
    s = light_half
    p1, i1 = quad((-s, light_h, -s), (s, light_h, -s), (s, light_h, s), (-s, light_h, s))
    m0, a0, e0 = _tri_params(2, (albedo,) * 3, (0, 0, 0), 0)
    m1, a1, e1 = _tri_params(2, (0, 0, 0), (le,) * 3, 0)
    scene = _pack([p0, p1], [i0, i1], [m0, m1], [a0, a1], [e0, e1], [(LAMBERT, 1.0, 1.5, 0.0)])
    cam = dict(eye=(0.0, 0.5, -3.0), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0),
               vfov_deg=45.0, width=width, height=height)
    return scene, cam


# --------------------------------------------------------------------------
# Procedural scenes: icospheres + tessellated boxes on a ground plane
# --------------------------------------------------------------------------
def procedural(seed=2, n_objects=2000, width=1920, height=1080, material_mode="lambert_conductor",
               n_material_ids=64, ground_albedo=0.5, light_le=20.0, attributes=False):
    """Half icospheres (level 3 or 4: 320 or 1280 faces), half boxes with an
    n x n grid per face (n in {3,4,5}: 108..300 triangles): expected
    1000 triangles per object on average.  Centres uniform in
    [-50,50] x [0,100] x [-50,50], scale log-uniform in [0.1, 5], a 400 x 400
    ground quad at y = 0 and 16 downward 10 x 10 quad lights at y = 120.

    material_mode:
      "lambert_conductor": per mesh, 50% Lambertian (albedo U[0.1,0.9]^3),
          50% GGX conductor (F0 U[0.1,0.9]^3, roughness U[0.05,0.8]).
      "divergence": per mesh one of ``n_material_ids`` ids drawn uniformly;
          ids in the first quarter are Lambertian, second conductor, third
          rough dielectric (ior U[1.3,1.8]), last quarter emissive Lambertian
          (albedo 0, emission 5 * U[0.2,1]^3).

    attributes=True adds shading attributes without changing the geometry:
    icospheres get their radial vertex normals (smooth shading), boxes zero
    normals (flat shading); every mesh gets texture coordinates (icospheres
    longitude/latitude, boxes (x + z, y) / scale, the ground (x, z) / 10);
    half of the Lambertian meshes a checker texture (frequency 2, 4 or 8,
    the ground 1) and half of the conductors become coated (coat roughness
    U[0, 0.5], ior U[1.3, 1.8]) over a base of the same albedo.  These
    choices come from a second generator (seed + 1000), so the scene's
    geometry and albedos equal those of attributes=False.
    """
    rng = np.random.default_rng(seed)
    rng2 = np.random.default_rng(seed + 1000)
    NRM, UV = [], []
    n_ico = n_objects // 2
    n_box = n_objects - n_ico
    P, I, M, A, E = [], [], [], [], []
    materials = [(LAMBERT, 1.0, 1.5, 0.0)]  # material 0: ground and lights

    if material_mode == "divergence":
        q = n_material_ids // 4
        mat_alb = rng.uniform(0.1, 0.9, size=(n_material_ids, 3))
        mat_emi = np.zeros((n_material_ids, 3))
        for mid in range(n_material_ids):
            if mid < q:
                materials.append((LAMBERT, 1.0, 1.5, 0.0))
            elif mid < 2 * q:
                materials.append((CONDUCTOR, float(rng.uniform(0.05, 0.8)), 1.5, 0.0))
            elif mid < 3 * q:
                materials.append((DIELECTRIC, float(rng.uniform(0.05, 0.8)), float(rng.uniform(1.3, 1.8)), 0.0))
            else:
                materials.append((LAMBERT, 1.0, 1.5, 0.0))
                mat_alb[mid] = 0.0
                mat_emi[mid] = 5.0 * rng.uniform(0.2, 1.0, size=3)

    def obj_material():
        if material_mode == "divergence":
            mid = int(rng.integers(0, n_material_ids))
            return mid + 1, mat_alb[mid], mat_emi[mid]
        if rng.uniform() < 0.5:
            alb = rng.uniform(0.1, 0.9, size=3)
            if attributes and rng2.uniform() < 0.5:
                materials.append((LAMBERT, 1.0, 1.5, float(rng2.choice([2.0, 4.0, 8.0]))))
                return len(materials) - 1, alb, np.zeros(3)
            return 0, alb, np.zeros(3)
        alb = rng.uniform(0.1, 0.9, size=3)
        rough = float(rng.uniform(0.05, 0.8))
        if attributes and rng2.uniform() < 0.5:
            materials.append((COATED, float(rng2.uniform(0.0, 0.5)), float(rng2.uniform(1.3, 1.8)), 0.0))
        else:
            materials.append((CONDUCTOR, rough, 1.5, 0.0))
        return len(materials) - 1, alb, np.zeros(3)

    centres = np.stack([rng.uniform(-50, 50, n_objects), rng.uniform(0, 100, n_objects),
                        rng.uniform(-50, 50, n_objects)], 1)
    scales = np.exp(rng.uniform(np.log(0.1), np.log(5.0), n_objects))
    kinds = np.array([0] * n_ico + [1] * n_box)
    rng.shuffle(kinds)
    for o in range(n_objects):
        c = centres[o]
        s = scales[o]
        if kinds[o] == 0:
            lvl = int(rng.integers(3, 5))
            up, ui = icosphere_unit(lvl)
            pos = c + s * up
            idx = ui
            NRM.append(up)
            UV.append(np.stack([np.arctan2(up[:, 2], up[:, 0]) / (2 * np.pi) + 0.5,
                                np.arccos(np.clip(up[:, 1], -1, 1)) / np.pi], 1))
        else:
            n = int(rng.integers(3, 6))
            ext = s * rng.uniform(0.5, 1.0, size=3)
            pos, idx = box_mesh(c - ext, c + ext, n)
            NRM.append(np.zeros_like(pos))
            UV.append(np.stack([(pos[:, 0] + pos[:, 2]) / s, pos[:, 1] / s], 1))
        mat, alb, emi = obj_material()
        P.append(pos)
        I.append(idx)
        m, a, e = _tri_params(idx.shape[0], alb, emi, mat)
        M.append(m)
        A.append(a)
        E.append(e)

    # ground
    gp, gi = quad((-200, 0, -200), (-200, 0, 200), (200, 0, 200), (200, 0, -200))
    gmat = 0
    if attributes:
        materials.append((LAMBERT, 1.0, 1.5, 1.0))
        gmat = len(materials) - 1
    m, a, e = _tri_params(2, (ground_albedo,) * 3, (0, 0, 0), gmat)
    P.append(gp); I.append(gi); M.append(m); A.append(a); E.append(e)
    NRM.append(np.zeros_like(gp)); UV.append(gp[:, [0, 2]] / 10.0)
    # 16 lights: 4 x 4 grid of 10 x 10 quads over [-45,45]^2 at y=120, facing -y
    for gx in np.linspace(-45, 45, 4):
        for gz in np.linspace(-45, 45, 4):
            lp, li = quad((gx - 5, 120, gz - 5), (gx + 5, 120, gz - 5), (gx + 5, 120, gz + 5), (gx - 5, 120, gz + 5))
            m, a, e = _tri_params(2, (0, 0, 0), (light_le,) * 3, 0)
            P.append(lp); I.append(li); M.append(m); A.append(a); E.append(e)
            NRM.append(np.zeros_like(lp)); UV.append(np.zeros((4, 2)))
    scene = _pack(P, I, M, A, E, materials)
    if attributes:
        scene["normals"] = np.ascontiguousarray(np.concatenate(NRM).astype(np.float32))
        scene["uvs"] = np.ascontiguousarray(np.concatenate(UV).astype(np.float32))
    cam = dict(eye=(0.0, 50.0, -130.0), target=(0.0, 40.0, 0.0), up=(0.0, 1.0, 0.0),
               vfov_deg=50.0, width=width, height=height)
    return scene, cam


# --------------------------------------------------------------------------
# Two-level scenes: meshes (ranges of the triangle list, object space) placed
# by instances (3x4 row-major object-to-world maps and their inverses)
# --------------------------------------------------------------------------
def affine(rot, scale, trans):
    """(o2w, w2o) as float32 [12] arrays for x -> scale * rot @ x + trans
    (rot orthonormal), the inverse computed in binary64 and rounded once."""
    rot = np.asarray(rot, np.float64)
    trans = np.asarray(trans, np.float64)
    A = scale * rot
    Ai = rot.T / scale
    o2w = np.concatenate([A, trans[:, None]], 1)
    w2o = np.concatenate([Ai, (-Ai @ trans)[:, None]], 1)
    return o2w.astype(np.float32).reshape(12), w2o.astype(np.float32).reshape(12)


def random_rotation(rng):
    """Uniform random rotation (quaternion with normal components)."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def split_into_instances(scene, parts):
    """A flat scene as a two-level one: its triangles cut into `parts`
    consecutive meshes, each placed once by the identity."""
    nt = scene["indices"].shape[0]
    cuts = np.linspace(0, nt, parts + 1).round().astype(np.int64)
    eye = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32)
    return {"mesh_first": cuts[:-1].astype(np.int32), "mesh_count": np.diff(cuts).astype(np.int32),
            "inst_mesh": np.arange(parts, dtype=np.int32), "o2w": np.tile(eye, (parts, 1)),
            "w2o": np.tile(eye, (parts, 1))}


def instanced_procedural(seed=6, n_instances=4000, n_meshes=32, width=1920, height=1080, ground_albedo=0.5,
                         light_le=20.0, attributes=False):
    """A scene of shared meshes: n_meshes object meshes (icospheres of level
    2-4 and tessellated boxes, unit size, each with its own material) placed
    n_instances times with random rotations, scales log-uniform in [0.1, 5]
    and centres uniform in [-50,50] x [0,100] x [-50,50]; a 400 x 400 ground
    quad (one instance) and a 10 x 10 downward quad light placed 16 times on a
    4 x 4 grid at y = 120 (the procedural scene's layout).  Materials per
    mesh: 50% Lambertian (albedo U[0.1,0.9]^3), 50% GGX conductor (F0
    U[0.1,0.9]^3, roughness U[0.05,0.8]).  attributes=True adds object-space
    vertex normals and texture coordinates, checker textures and coats as in
    procedural (from a second generator: same geometry and placements).
    Returns (scene, instances, cam)."""
    rng = np.random.default_rng(seed)
    rng2 = np.random.default_rng(seed + 1000)
    P, I, M, A, E = [], [], [], [], []
    NRM, UV = [], []
    materials = [(LAMBERT, 1.0, 1.5, 0.0)]
    first, count = [], []
    nt = 0

    def add(pos, idx, mat, alb, emi, nrm=None, uv=None):
        nonlocal nt
        P.append(pos); I.append(idx)
        NRM.append(np.zeros_like(pos) if nrm is None else nrm)
        UV.append(np.zeros((pos.shape[0], 2)) if uv is None else uv)
        m, a, e = _tri_params(idx.shape[0], alb, emi, mat)
        M.append(m); A.append(a); E.append(e)
        first.append(nt); count.append(idx.shape[0])
        nt += idx.shape[0]

    for k in range(n_meshes):
        if k % 2 == 0:
            pos, idx = icosphere_unit(int(rng.integers(2, 5)))
            nrm = pos
            uv = np.stack([np.arctan2(pos[:, 2], pos[:, 0]) / (2 * np.pi) + 0.5,
                           np.arccos(np.clip(pos[:, 1], -1, 1)) / np.pi], 1)
        else:
            pos, idx = box_mesh(-rng.uniform(0.5, 1.0, 3), rng.uniform(0.5, 1.0, 3), int(rng.integers(2, 6)))
            nrm = None
            uv = np.stack([pos[:, 0] + pos[:, 2], pos[:, 1]], 1)
        alb = rng.uniform(0.1, 0.9, size=3)
        if rng.uniform() < 0.5:
            mat = 0
            if attributes and rng2.uniform() < 0.5:
                materials.append((LAMBERT, 1.0, 1.5, float(rng2.choice([2.0, 4.0, 8.0]))))
                mat = len(materials) - 1
        else:
            rough = float(rng.uniform(0.05, 0.8))
            if attributes and rng2.uniform() < 0.5:
                materials.append((COATED, float(rng2.uniform(0.0, 0.5)), float(rng2.uniform(1.3, 1.8)), 0.0))
            else:
                materials.append((CONDUCTOR, rough, 1.5, 0.0))
            mat = len(materials) - 1
        add(pos, idx, mat, alb, np.zeros(3), nrm, uv)
    gp, gi = quad((-200, 0, -200), (-200, 0, 200), (200, 0, 200), (200, 0, -200))
    gmat = 0
    if attributes:
        materials.append((LAMBERT, 1.0, 1.5, 1.0))
        gmat = len(materials) - 1
    add(gp, gi, gmat, (ground_albedo,) * 3, (0, 0, 0), None, gp[:, [0, 2]] / 10.0)
    lp, li = quad((-5, 0, -5), (5, 0, -5), (5, 0, 5), (-5, 0, 5))
    add(lp, li, 0, (0, 0, 0), (light_le,) * 3)
    ground, light = n_meshes, n_meshes + 1
    inst_mesh, o2w, w2o = [], [], []
    for q in range(n_instances):
        a, b = affine(random_rotation(rng), float(np.exp(rng.uniform(np.log(0.1), np.log(5.0)))),
                      (rng.uniform(-50, 50), rng.uniform(0, 100), rng.uniform(-50, 50)))
        inst_mesh.append(int(rng.integers(0, n_meshes))); o2w.append(a); w2o.append(b)
    a, b = affine(np.eye(3), 1.0, (0, 0, 0))
    inst_mesh.append(ground); o2w.append(a); w2o.append(b)
    for gx in np.linspace(-45, 45, 4):
        for gz in np.linspace(-45, 45, 4):
            a, b = affine(np.eye(3), 1.0, (gx, 120.0, gz))
            inst_mesh.append(light); o2w.append(a); w2o.append(b)
    scene = _pack(P, I, M, A, E, materials)
    if attributes:
        scene["normals"] = np.ascontiguousarray(np.concatenate(NRM).astype(np.float32))
        scene["uvs"] = np.ascontiguousarray(np.concatenate(UV).astype(np.float32))
    inst = {"mesh_first": np.array(first, np.int32), "mesh_count": np.array(count, np.int32),
            "inst_mesh": np.array(inst_mesh, np.int32), "o2w": np.array(o2w, np.float32),
            "w2o": np.array(w2o, np.float32)}
    cam = dict(eye=(0.0, 50.0, -130.0), target=(0.0, 40.0, 0.0), up=(0.0, 1.0, 0.0),
               vfov_deg=50.0, width=width, height=height)
    return scene, inst, cam


def flatten_instances(scene, inst):
    """The world-space flat scene of a two-level one (every instance's
    triangles mapped by its o2w in binary64, rounded once; per-triangle
    parameters copied), for size and speed comparisons."""
    pos = scene["positions"].astype(np.float64)
    idx = scene["indices"]
    P, I, M, A, E = [], [], [], [], []
    for q, m in enumerate(inst["inst_mesh"]):
        f, n = int(inst["mesh_first"][m]), int(inst["mesh_count"][m])
        if n == 0:
            continue
        T = inst["o2w"][q].astype(np.float64).reshape(3, 4)
        tri = idx[f:f + n]
        v = pos[tri.reshape(-1)] @ T[:, :3].T + T[:, 3]
        P.append(v)
        I.append(np.arange(3 * n, dtype=np.int32).reshape(n, 3))
        M.append(scene["tri_mat"][f:f + n]); A.append(scene["albedo"][f:f + n]); E.append(scene["emission"][f:f + n])
    return _pack(P, I, M, A, E, scene["materials"], sky=scene["sky"])


def random_soup(seed, n_tris, extent=1.0, emissive_frac=0.1, materials=None):
    """Random triangle soup in [-extent, extent]^3 (tiny scenes for
    intersection and parity tests), with shared edges from a small vertex
    pool so that edge and vertex hits occur."""
    rng = np.random.default_rng(seed)
    nv = max(3, n_tris // 2 + 3)
    pos = rng.uniform(-extent, extent, size=(nv, 3))
    # snap some coordinates onto a coarse grid to create axis-aligned and
    # coplanar configurations
    snap = rng.uniform(size=pos.shape) < 0.3
    pos[snap] = np.round(pos[snap] * 4) / 4
    idx = np.empty((n_tris, 3), np.int32)
    for t in range(n_tris):
        idx[t] = rng.choice(nv, 3, replace=False)
    mats = materials if materials is not None else [(LAMBERT, 1.0, 1.5, 0.0)]
    tri_mat = rng.integers(0, len(mats), n_tris).astype(np.int32)
    alb = rng.uniform(0.1, 0.9, size=(n_tris, 3))
    emi = np.zeros((n_tris, 3))
    ne = int(round(emissive_frac * n_tris))
    if ne:
        sel = rng.choice(n_tris, ne, replace=False)
        emi[sel] = rng.uniform(0.5, 5.0, size=(ne, 3))
    return _pack([pos], [idx], [tri_mat], [alb], [emi], mats)


def batch_jobs(seed=4, n_jobs=64, tri_lo=1e4, tri_hi=2e6):
    """Job list of the batched workload: per job a scene seed, a triangle
    count T drawn log-uniform in [tri_lo, tri_hi] (objects = T / 500: the
    procedural mix averages 500 triangles per object), a resolution from
    {256^2, 512^2, 1024^2, 1920x1080} and 1..8 spp."""
    rng = np.random.default_rng(seed)
    res = [(256, 256), (512, 512), (1024, 1024), (1920, 1080)]
    jobs = []
    for j in range(n_jobs):
        t = float(np.exp(rng.uniform(np.log(tri_lo), np.log(tri_hi))))
        w, h = res[int(rng.integers(0, 4))]
        spp = int(rng.integers(1, 9))
        jobs.append(dict(scene_seed=1000 + j, n_objects=max(2, int(round(t / 500.0))),
                         width=w, height=h, spp=spp))
    return jobs


def perturb_albedo(albedo, seed=5, sigma=0.05, lo=0.02, hi=0.95):
    """Per-triangle albedo + N(0, sigma), clipped to [lo, hi]."""
    rng = np.random.default_rng(seed)
    out = albedo.astype(np.float64) + rng.normal(0.0, sigma, size=albedo.shape)
    return np.clip(out, lo, hi).astype(np.float32)


def pixel_subset(width, height, n, seed=1234):
    """Sorted seeded subset of pixel ids (py * width + px)."""
    rng = np.random.default_rng(seed)
    n = min(n, width * height)
    return np.sort(rng.choice(width * height, n, replace=False)).astype(np.int32)
