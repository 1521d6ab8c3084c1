"""CPU checks of the C-ABI library: it loads, exports every function the
header declares, validates its inputs, and builds a well-formed BVH4 with
the same light set and CDF as the oracle (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2605_27323_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ptmi = pytest.importorskip("paper_2605_27323_amd.ptmi")


def header_functions():
    txt = open(os.path.join(ROOT, "include", "ptmi.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_header_function():
    L = ptmi.lib()
    names = header_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    # the binding declares exactly these
    assert set(names) == set(ptmi.SIGNATURES)


def test_create_without_gpu_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    rc = ptmi.lib().pt_create(C.byref(h), 0)
    assert rc == ptmi.PT_EHIP
    assert len(ptmi.lib().pt_last_error()) > 0


def _desc(scene):
    keep = {k: np.ascontiguousarray(v) for k, v in scene.items()}
    d = ptmi.SceneDesc(keep["positions"].shape[0], keep["indices"].shape[0], keep["materials"].shape[0],
                       keep["positions"].ctypes.data, keep["indices"].ctypes.data, keep["tri_mat"].ctypes.data,
                       keep["materials"].ctypes.data, keep["albedo"].ctypes.data, keep["emission"].ctypes.data,
                       (C.c_float * 3)(*keep["sky"].tolist()))
    return d, keep


def test_invalid_inputs_rejected():
    L = ptmi.lib()
    h = C.c_void_p()
    assert L.pt_create(C.byref(h), -1) == 0
    scene, cam = scenes.cornell()
    bad = {k: v.copy() for k, v in scene.items()}
    bad["indices"][3, 1] = 10_000
    d, keep = _desc(bad)
    assert L.pt_load_scene(h, C.byref(d)) == ptmi.PT_EINVAL
    bad = {k: v.copy() for k, v in scene.items()}
    bad["positions"][5, 2] = np.nan
    d, keep = _desc(bad)
    assert L.pt_load_scene(h, C.byref(d)) == ptmi.PT_EINVAL
    bad = {k: v.copy() for k, v in scene.items()}
    bad["materials"] = np.array([[7, 0.5, 1.5, 0]], np.float32)
    d, keep = _desc(bad)
    assert L.pt_load_scene(h, C.byref(d)) == ptmi.PT_EINVAL
    bad = {k: v.copy() for k, v in scene.items()}
    bad["emission"][0, 0] = -1
    d, keep = _desc(bad)
    assert L.pt_load_scene(h, C.byref(d)) == ptmi.PT_EINVAL
    # build before load, render on a host-only context, null pointers
    info = ptmi.BvhInfo()
    assert L.pt_build_bvh(h, None, C.byref(info)) == ptmi.PT_ESTATE
    d, keep = _desc(scene)
    assert L.pt_load_scene(h, C.byref(d)) == 0
    assert L.pt_build_bvh(h, None, C.byref(info)) == 0
    a = ptmi.RenderArgs(1, 1, 0, 0, 0, 1, -1, 0, 0, 0, 0)
    assert L.pt_render_frame(h, C.byref(a), None, None, None, 0, None) == ptmi.PT_ESTATE
    assert L.pt_load_scene(h, None) == ptmi.PT_EINVAL
    camd = ptmi.Camera((C.c_double * 3)(0, 0, 0), (C.c_double * 3)(0, 0, 0), (C.c_double * 3)(0, 1, 0), 40.0, 8, 8)
    assert L.pt_set_camera(h, C.byref(camd)) == ptmi.PT_EINVAL  # eye == target
    camd = ptmi.Camera((C.c_double * 3)(0, 0, 0), (C.c_double * 3)(0, 0, 1), (C.c_double * 3)(0, 1, 0), 200.0, 8, 8)
    assert L.pt_set_camera(h, C.byref(camd)) == ptmi.PT_EINVAL  # fov
    opts = ptmi.BvhOpts(9, 0)
    assert L.pt_build_bvh(h, C.byref(opts), C.byref(info)) == ptmi.PT_EINVAL
    assert L.pt_destroy(h) == 0


def _walk(nodes, nt):
    """Decode the BVH4 (test-side reader of the node layout: origin, scale
    exponents, binary16 plane offsets, references): returns leaf ranges and,
    per leaf, the chain of ancestor boxes, decoded exactly in float64."""
    f = nodes.view(np.float32).reshape(-1, 20)
    u = nodes.view(np.uint32).reshape(-1, 20)
    h = nodes.view(np.float16).reshape(-1, 40)
    leaves = []
    depth = 0
    stack = [(0, [], 1)]
    while stack:
        ni, boxes, lvl = stack.pop()
        depth = max(depth, lvl)
        org = f[ni, 0:3].astype(np.float64)
        scale = np.array([2.0 ** (((int(u[ni, 3]) >> (8 * a)) & 255) - 128) for a in range(3)])
        for c in range(4):
            ref = int(u[ni, 16 + c])
            # axis a: halves 8 + 8a .. 8 + 8a + 7 = lower planes of children 0..3, upper planes of 0..3
            hl = np.array([h[ni, 8 + 8 * a + c] for a in range(3)], np.float64)
            hh = np.array([h[ni, 8 + 8 * a + 4 + c] for a in range(3)], np.float64)
            if ref == 0xFFFFFFFF:
                assert np.isposinf(hl).all() and np.isneginf(hh).all()
                continue
            lo = org + hl * scale
            hi = org + hh * scale
            if ref & 0x80000000:
                first = ref & ((1 << 27) - 1)
                cnt = ((ref >> 27) & 15) + 1
                leaves.append((first, cnt, boxes + [(lo, hi)]))
            else:
                assert 0 < ref < nodes.shape[0]
                stack.append((ref, boxes + [(lo, hi)], lvl + 1))
    return leaves, depth


@pytest.mark.parametrize("max_leaf", [1, 4, 8])
@pytest.mark.parametrize("which", ["cornell", "procedural", "soup", "single", "empty"])
def test_bvh4_structure(which, max_leaf):
    if which == "cornell":
        scene, _ = scenes.cornell()
    elif which == "procedural":
        scene, _ = scenes.procedural(seed=3, n_objects=30)
    elif which == "soup":
        scene = scenes.random_soup(5, 300, emissive_frac=0.2)
    elif which == "single":
        scene = scenes.random_soup(6, 1, emissive_frac=1.0)
    else:
        scene = scenes.random_soup(7, 1)
        scene = dict(scene, indices=np.zeros((0, 3), np.int32), tri_mat=np.zeros(0, np.int32),
                     albedo=np.zeros((0, 3), np.float32), emission=np.zeros((0, 3), np.float32))
    ctx = ptmi.Context(scene, device=-1, max_leaf=max_leaf)
    nodes, tris, lights = ctx.host_bvh()
    nt = scene["indices"].shape[0]
    leaves, depth = _walk(nodes, nt)
    assert depth == ctx.info.depth
    assert ctx.info.stack_entries == 3 * depth + 1
    covered = np.zeros(nt, int)
    ids = tris[:, 3].view(np.uint32) if nt else np.zeros(0, np.uint32)
    pos = scene["positions"]
    idx = scene["indices"]
    for first, cnt, boxes in leaves:
        assert cnt <= max_leaf
        for j in range(first, first + cnt):
            covered[j] += 1
            tid = int(ids[j])
            v = pos[idx[tid]].astype(np.float32)
            assert np.array_equal(tris[j, [0, 1, 2]], v[0])
            assert np.array_equal(tris[j, [4, 5, 6]], v[1])
            assert np.array_equal(tris[j, [8, 9, 10]], v[2])
            for lo, hi in boxes:  # every ancestor box encloses the triangle
                assert (v >= lo).all() and (v <= hi).all()
    assert (covered == 1).all()
    if nt:
        assert sorted(ids.tolist()) == list(range(nt))
        minfo = tris[:, 7].view(np.uint32)
        assert np.array_equal(minfo & 0x7FFFFFFF, scene["tri_mat"][ids])
        is_light = (scene["emission"] > 0).any(1)
        assert np.array_equal((minfo >> 31).astype(bool), is_light[ids])


def test_light_cdf_matches_oracle():
    scene = scenes.random_soup(11, 200, emissive_frac=0.3)
    ctx = ptmi.Context(scene, device=-1)
    _, tris, lights = ctx.host_bvh()
    S = oracle.Scene(scene, bvh=False)
    assert lights.shape[0] == S.num_lights
    ids = tris[:, 3].view(np.uint32)
    light_ids = ids[lights[:, 0]]
    assert (np.diff(light_ids.astype(np.int64)) > 0).all()  # input order
    assert np.array_equal(lights[:, 2], light_ids) and not lights[:, 3].any()
    rng = np.random.default_rng(0)
    words = np.concatenate([rng.integers(0, 2**32, 5000, dtype=np.uint64),
                            lights[:, 1].astype(np.uint64), (lights[:-1, 1].astype(np.uint64) + 1)])
    for w in words:
        j_lib = int(np.searchsorted(lights[:, 1], np.uint32(w), side="left"))
        assert j_lib == S.pick_light(int(w))


@pytest.mark.parametrize("which", ["procedural", "soup", "degenerate"])
def test_largest_triangles_marked(which):
    # the triangle records mark the 64 triangles of largest area (ties to
    # the smaller input id, zero area never) with their slot + 1 in the
    # last word; the adjoint sums those triangles' gradients per workgroup
    if which == "procedural":
        scene, _ = scenes.procedural(seed=3, n_objects=30)
    elif which == "soup":
        scene = scenes.random_soup(5, 40, emissive_frac=0.2)
    else:
        from tests._parity import degenerate_scene
        scene, _ = degenerate_scene()
    ctx = ptmi.Context(scene, device=-1)
    _, tris, _ = ctx.host_bvh()
    P = scene["positions"].astype(np.float64)[scene["indices"]]
    c = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    a2 = (c * c).sum(1)
    order = sorted((i for i in range(len(a2)) if a2[i] > 0), key=lambda i: (-a2[i], i))[:64]
    ids = tris[:, 3].view(np.uint32)
    slot = np.zeros(len(a2), np.int64)
    slot[ids] = tris[:, 11].view(np.uint32)
    expect = np.zeros(len(a2), np.int64)
    for k, i in enumerate(order):
        expect[i] = k + 1
    assert np.array_equal(slot, expect)


def test_attributes_validated():
    L = ptmi.lib()
    h = C.c_void_p()
    assert L.pt_create(C.byref(h), -1) == 0
    scene, _ = scenes.cornell_attributes()
    nv = scene["positions"].shape[0]
    nrm = np.ascontiguousarray(scene["normals"])
    uvs = np.ascontiguousarray(scene["uvs"])
    a = ptmi.AttributesDesc(nv, nrm.ctypes.data, uvs.ctypes.data)
    assert L.pt_set_attributes(h, C.byref(a)) == ptmi.PT_ESTATE  # no scene yet
    d, keep = _desc(scene)
    assert L.pt_load_scene(h, C.byref(d)) == 0
    bad = ptmi.AttributesDesc(nv - 1, nrm.ctypes.data, None)
    assert L.pt_set_attributes(h, C.byref(bad)) == ptmi.PT_EINVAL  # count mismatch
    nan = nrm.copy()
    nan[3, 1] = np.inf
    bad = ptmi.AttributesDesc(nv, nan.ctypes.data, None)
    assert L.pt_set_attributes(h, C.byref(bad)) == ptmi.PT_EINVAL
    # a coat needs a finite ior > 0; the checker frequency must be finite and >= 0
    for m in ([3, 0.2, 0.0, 0], [0, 1.0, 1.5, -1.0], [0, 1.0, 1.5, np.nan]):
        b = {k: v.copy() for k, v in scene.items()}
        b["materials"] = np.array([m], np.float32)
        b["tri_mat"][:] = 0
        db, kb = _desc(b)
        assert L.pt_load_scene(h, C.byref(db)) == ptmi.PT_EINVAL, m
    assert L.pt_load_scene(h, C.byref(d)) == 0
    assert L.pt_set_attributes(h, C.byref(a)) == 0
    info = ptmi.BvhInfo()
    assert L.pt_build_bvh(h, None, C.byref(info)) == 0
    nt = scene["indices"].shape[0]
    assert info.attribute_bytes == 64 * nt
    # one record per triangle record
    tris = np.zeros((nt, 12), np.float32)
    assert L.pt_get_bvh(h, None, tris.ctypes.data, None, None) == 0
    ids = tris[:, 3].view(np.uint32)
    assert sorted(ids.tolist()) == list(range(nt))
    # NULL desc removes the attributes; the scene reports none
    assert L.pt_set_attributes(h, None) == 0
    assert L.pt_build_bvh(h, None, C.byref(info)) == 0
    assert info.attribute_bytes == 0
    assert L.pt_destroy(h) == 0


def test_keep_hits_workspace_adds_vertex_records():
    # PT_FLAG_KEEP_HITS reserves, per path sample and vertex (max_depth + 1
    # of them), an 8-byte hit record and a 1-byte visibility, each region
    # 256-byte aligned; forward workspaces do not change
    L = ptmi.lib()
    h = C.c_void_p()
    assert L.pt_create(C.byref(h), -1) == 0
    scene, cam = scenes.cornell()
    d, keep = _desc(scene)
    info = ptmi.BvhInfo()
    assert L.pt_load_scene(h, C.byref(d)) == 0
    assert L.pt_build_bvh(h, None, C.byref(info)) == 0
    W, H = 33, 17
    camd = ptmi.Camera((C.c_double * 3)(*cam["eye"]), (C.c_double * 3)(*cam["target"]), (C.c_double * 3)(*cam["up"]),
                       float(cam["vfov_deg"]), W, H)
    assert L.pt_set_camera(h, C.byref(camd)) == 0

    def up(x):
        return (x + 255) // 256 * 256

    for mode in (ptmi.MODE_MEGA, ptmi.MODE_WAVE):
        for spp, depth in ((3, 5), (1, 0), (2, 12)):
            sizes = {}
            for flags in (0, ptmi.FLAG_KEEP_HITS):
                a = ptmi.RenderArgs(spp, depth, 0, 0, 0, 1, -1, mode, flags, 0, 0)
                for fn, key in ((L.pt_backward_workspace_size, "b"), (L.pt_workspace_size, "f")):
                    n = C.c_uint64()
                    assert fn(h, C.byref(a), C.byref(n)) == 0
                    sizes[(flags, key)] = n.value
            nrec = W * H * spp * (depth + 1)
            assert sizes[(ptmi.FLAG_KEEP_HITS, "b")] - sizes[(0, "b")] == up(8 * nrec) + up(nrec)
            assert sizes[(ptmi.FLAG_KEEP_HITS, "f")] == sizes[(0, "f")]
    assert L.pt_destroy(h) == 0
