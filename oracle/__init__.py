"""ctypes wrapper of the CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg; the renderer never calls into it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")


def default_threads():
    """Host threads of an oracle call: the CPUs this process may run on,
    capped by OMP_NUM_THREADS when it is set (a shared host's share)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cap = os.environ.get("OMP_NUM_THREADS", "")
    if cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(HERE, "liboracle.so")
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    L = C.CDLL(path)
    L.orc_scene_create.restype = C.c_void_p
    L.orc_scene_create.argtypes = [C.c_int32, f32p, C.c_int32, i32p, i32p, C.c_int32, f32p, f32p, f32p,
                                   f32p, C.c_int32]
    L.orc_scene_destroy.argtypes = [C.c_void_p]
    L.orc_scene_set_params.argtypes = [C.c_void_p, f32p, f32p]
    L.orc_scene_num_lights.argtypes = [C.c_void_p]
    L.orc_scene_num_lights.restype = C.c_int32
    L.orc_scene_bvh_stats.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    d3 = np.ctypeslib.ndpointer(np.float64, shape=(3,), flags="C_CONTIGUOUS")
    L.orc_camera.argtypes = [d3, d3, d3, C.c_double, C.c_int32, C.c_int32, f32p]
    L.orc_philox4x64.argtypes = [u64p, u64p, u64p]
    L.orc_render.restype = C.c_int32
    L.orc_render.argtypes = [C.c_void_p, f32p, C.c_int32, C.c_int32, i32p, C.c_int32, C.c_int32, C.c_int32,
                             C.c_uint64, C.c_uint32, C.c_uint32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                             C.c_int32, f32p, C.c_void_p, C.c_void_p]
    L.orc_backward.restype = C.c_int32
    L.orc_backward.argtypes = [C.c_void_p, f32p, C.c_int32, C.c_int32, i32p, C.c_int32, C.c_int32, C.c_int32,
                               C.c_uint64, C.c_uint32, C.c_uint32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                               f32p, f64p, f64p, C.c_void_p, C.c_void_p]
    L.orc_radical_inverse.restype = C.c_float
    L.orc_radical_inverse.argtypes = [C.c_uint32, C.c_int32]
    L.orc_halton_jitter.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, f32p]
    L.orc_closest.argtypes = [C.c_void_p, C.c_int32, f32p, f32p, C.c_float, C.c_int32, f32p, i32p, f32p, f32p,
                              C.c_void_p]
    L.orc_scene_set_instances.restype = C.c_int32
    L.orc_scene_set_instances.argtypes = [C.c_void_p, C.c_int32, i32p, i32p, C.c_int32, i32p, f32p, f32p]
    L.orc_anyhit.argtypes = [C.c_void_p, C.c_int32, f32p, f32p, C.c_float, C.c_int32, u8p]
    L.orc_tri_test.restype = C.c_int32
    L.orc_tri_test.argtypes = [f32p, f32p, f32p, f32p, f32p, C.POINTER(C.c_float), C.POINTER(C.c_float),
                               C.POINTER(C.c_float)]
    L.orc_bsdf_eval.argtypes = [C.c_int32, C.c_float, C.c_float, C.c_float, f32p, f32p, f32p, f32p, f32p,
                                C.POINTER(C.c_float)]
    L.orc_bsdf_sample.restype = C.c_int32
    L.orc_bsdf_sample.argtypes = [C.c_int32, C.c_float, C.c_float, C.c_float, f32p, f32p, f32p, C.c_float,
                                  C.c_float, C.c_float, f32p, f32p, C.POINTER(C.c_float)]
    L.orc_scene_set_attributes.restype = C.c_int32
    L.orc_scene_set_attributes.argtypes = [C.c_void_p, C.c_int32, i32p, C.c_void_p, C.c_void_p]
    L.orc_shading_normal.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_float, C.c_float, f32p]
    L.orc_texture.restype = C.c_float
    L.orc_texture.argtypes = [C.c_void_p, C.c_int32, C.c_float, C.c_float, C.c_float]
    L.orc_sample_triangle.argtypes = [f32p, f32p, f32p, C.c_float, C.c_float, f32p]
    L.orc_offset.argtypes = [f32p, f32p, f32p, f32p]
    L.orc_frame.argtypes = [f32p, f32p, f32p]
    L.orc_pick_light.restype = C.c_int32
    L.orc_pick_light.argtypes = [C.c_void_p, C.c_uint32]
    L.orc_unif.restype = C.c_float
    L.orc_unif.argtypes = [C.c_uint32]
    _LIB = L
    return L


def _f32(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return a


def camera(cam):
    """Binary32 camera constants E, R, U, F as a (12,) array."""
    out = np.zeros(12, np.float32)
    lib().orc_camera(np.asarray(cam["eye"], np.float64), np.asarray(cam["target"], np.float64),
                     np.asarray(cam["up"], np.float64), float(cam["vfov_deg"]), int(cam["width"]),
                     int(cam["height"]), out)
    return out


def philox4x64(ctr, key):
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64(np.asarray(ctr, np.uint64), np.asarray(key, np.uint64), out)
    return out


def unif(w):
    return lib().orc_unif(int(w))


class Scene:
    """Oracle-side scene (own triangle copy, own light CDF, own BVH)."""

    def __init__(self, scene, bvh=True, instances=None):
        """instances (optional): a two-level scene, dict of mesh_first,
        mesh_count (int32 [n_meshes]), inst_mesh (int32 [n_inst]), o2w and
        w2o (float32 [n_inst, 12], 3x4 row-major); the scene's triangles are
        then the meshes, in object space."""
        L = lib()
        pos = _f32(scene["positions"]).reshape(-1)
        idx = np.ascontiguousarray(scene["indices"], np.int32).reshape(-1)
        self.nt = idx.size // 3
        self.ptr = L.orc_scene_create(pos.size // 3, pos, self.nt, idx,
                                      np.ascontiguousarray(scene["tri_mat"], np.int32),
                                      scene["materials"].shape[0], _f32(scene["materials"]).reshape(-1),
                                      _f32(scene["albedo"]).reshape(-1), _f32(scene["emission"]).reshape(-1),
                                      _f32(scene["sky"]), 1 if bvh else 0)
        if not self.ptr:
            raise ValueError("oracle rejected the scene")
        self.has_bvh = bool(bvh)
        nrm, uvs = scene.get("normals"), scene.get("uvs")
        if nrm is not None or uvs is not None:
            self._nrm = None if nrm is None else _f32(nrm).reshape(-1)
            self._uvs = None if uvs is None else _f32(uvs).reshape(-1)
            rc = L.orc_scene_set_attributes(
                self.ptr, pos.size // 3, idx,
                None if self._nrm is None else self._nrm.ctypes.data_as(C.c_void_p),
                None if self._uvs is None else self._uvs.ctypes.data_as(C.c_void_p))
            if rc != 0:
                raise ValueError("oracle rejected the vertex attributes")
        if instances is not None:
            i = instances
            rc = L.orc_scene_set_instances(self.ptr, len(i["mesh_first"]),
                                           np.ascontiguousarray(i["mesh_first"], np.int32),
                                           np.ascontiguousarray(i["mesh_count"], np.int32), len(i["inst_mesh"]),
                                           np.ascontiguousarray(i["inst_mesh"], np.int32),
                                           _f32(i["o2w"]).reshape(-1), _f32(i["w2o"]).reshape(-1))
            if rc != 0:
                raise ValueError("oracle rejected the instances")

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().orc_scene_destroy(self.ptr)
            self.ptr = None

    def set_params(self, albedo, emission):
        lib().orc_scene_set_params(self.ptr, _f32(albedo).reshape(-1), _f32(emission).reshape(-1))

    @property
    def num_lights(self):
        return lib().orc_scene_num_lights(self.ptr)

    def bvh_stats(self):
        n, d = C.c_int32(), C.c_int32()
        lib().orc_scene_bvh_stats(self.ptr, C.byref(n), C.byref(d))
        return n.value, d.value

    def pick_light(self, w):
        return lib().orc_pick_light(self.ptr, int(w))

    def shading_normal(self, tri, b1, b2, inst=0):
        """Shading normal of triangle tri (of instance inst) at (b1, b2)."""
        out = np.zeros(3, np.float32)
        lib().orc_shading_normal(self.ptr, int(inst), int(tri), float(b1), float(b2), out)
        return out

    def texture(self, tri, b1, b2, freq):
        """Checker factor of the albedo at (b1, b2) of triangle tri."""
        return lib().orc_texture(self.ptr, int(tri), float(b1), float(b2), float(freq))

    def render(self, cam, pixels=None, spp=1, max_depth=5, seed=0, frame=0, job=0, nee=True,
               rr_start=-1, use_bvh=None, threads=None, per_sample=False, sampler=0):
        """Returns (rgb [n,3], fragile [n] bool[, per-sample L [n, spp, 3]])."""
        W, H = int(cam["width"]), int(cam["height"])
        if pixels is None:
            pixels = np.arange(W * H, dtype=np.int32)
        pixels = np.ascontiguousarray(pixels, np.int32)
        n = pixels.size
        out = np.zeros((n, 3), np.float32)
        frag = np.zeros(n, np.uint8)
        ps = np.zeros((n, spp, 3), np.float32) if per_sample else None
        if use_bvh is None:
            use_bvh = self.has_bvh
        if threads is None:
            threads = default_threads()
        rc = lib().orc_render(self.ptr, camera(cam), W, H, pixels, n, int(spp), int(max_depth), int(seed),
                              int(frame), int(job), int(bool(nee)), int(rr_start), int(sampler), int(use_bvh),
                              int(threads), out.reshape(-1), frag.ctypes.data,
                              ps.ctypes.data if ps is not None else None)
        if rc != 0:
            raise ValueError(f"orc_render failed ({rc})")
        if per_sample:
            return out, frag, ps
        return out, frag

    def backward(self, cam, d_image, pixels=None, spp=1, max_depth=5, seed=0, frame=0, job=0, nee=True,
                 use_bvh=None, threads=None, sampler=0):
        """Returns (g_albedo [nt,3], g_emission [nt,3], abs_albedo, abs_emission), binary64."""
        W, H = int(cam["width"]), int(cam["height"])
        if pixels is None:
            pixels = np.arange(W * H, dtype=np.int32)
        pixels = np.ascontiguousarray(pixels, np.int32)
        d_image = _f32(d_image).reshape(-1)
        assert d_image.size == pixels.size * 3
        ga = np.zeros(self.nt * 3, np.float64)
        ge = np.zeros(self.nt * 3, np.float64)
        aa = np.zeros(self.nt * 3, np.float64)
        ae = np.zeros(self.nt * 3, np.float64)
        if use_bvh is None:
            use_bvh = self.has_bvh
        if threads is None:
            threads = default_threads()
        rc = lib().orc_backward(self.ptr, camera(cam), W, H, pixels, pixels.size, int(spp), int(max_depth),
                                int(seed), int(frame), int(job), int(bool(nee)), int(sampler), int(use_bvh),
                                int(threads), d_image, ga, ge, aa.ctypes.data, ae.ctypes.data)
        if rc != 0:
            raise ValueError(f"orc_backward failed ({rc})")
        return ga.reshape(-1, 3), ge.reshape(-1, 3), aa.reshape(-1, 3), ae.reshape(-1, 3)

    def closest(self, o, d, tmax=np.inf, mode=1, with_inst=False):
        o = _f32(o).reshape(-1)
        d = _f32(d).reshape(-1)
        n = o.size // 3
        t = np.zeros(n, np.float32)
        prim = np.zeros(n, np.int32)
        b1 = np.zeros(n, np.float32)
        b2 = np.zeros(n, np.float32)
        inst = np.zeros(n, np.int32)
        lib().orc_closest(self.ptr, n, o, d, float(tmax), int(mode), t, prim, b1, b2, inst.ctypes.data)
        if with_inst:
            return t, prim, b1, b2, inst
        return t, prim, b1, b2

    def anyhit(self, o, d, tmax, mode=1):
        o = _f32(o).reshape(-1)
        d = _f32(d).reshape(-1)
        n = o.size // 3
        occ = np.zeros(n, np.uint8)
        lib().orc_anyhit(self.ptr, n, o, d, float(tmax), int(mode), occ)
        return occ.astype(bool)


def radical_inverse(n, base):
    """phi_base(n) truncated to 24 bits (base 2 or 3)."""
    if base not in (2, 3):
        raise ValueError("the sampler's radical inverse has bases 2 and 3")
    return lib().orc_radical_inverse(int(n), int(base))


def halton_jitter(seed, pixel, sample, job=0):
    """Camera jitter (u0, u1) of the Halton(2,3) sampler with the pixel's rotation."""
    out = np.zeros(2, np.float32)
    lib().orc_halton_jitter(int(seed), int(pixel), int(sample), int(job), out)
    return float(out[0]), float(out[1])


def tri_test(o, d, v0, v1, v2):
    t, b1, b2 = C.c_float(), C.c_float(), C.c_float()
    hit = lib().orc_tri_test(_f32(o), _f32(d), _f32(v0), _f32(v1), _f32(v2), C.byref(t), C.byref(b1), C.byref(b2))
    return bool(hit), t.value, b1.value, b2.value


def bsdf_eval(mtype, rough, alb, n, wo, wi, ior=1.5, tex=1.0):
    f = np.zeros(3, np.float32)
    pdf = C.c_float()
    lib().orc_bsdf_eval(int(mtype), float(rough), float(ior), float(tex), _f32(alb), _f32(n), _f32(wo), _f32(wi),
                        f, C.byref(pdf))
    return f, pdf.value


def bsdf_sample(mtype, rough, ior, alb, n, wo, u4, u5, u6, tex=1.0):
    wi = np.zeros(3, np.float32)
    w = np.zeros(3, np.float32)
    pdf = C.c_float()
    ok = lib().orc_bsdf_sample(int(mtype), float(rough), float(ior), float(tex), _f32(alb), _f32(n), _f32(wo),
                               float(u4), float(u5), float(u6), wi, w, C.byref(pdf))
    return bool(ok), wi, w, pdf.value


def sample_triangle(v0, v1, v2, u1, u2):
    out = np.zeros(3, np.float32)
    lib().orc_sample_triangle(_f32(v0), _f32(v1), _f32(v2), float(u1), float(u2), out)
    return out


def frame(n):
    """Tangent and bitangent of the BSDF frame around the unit normal n."""
    t = np.zeros(3, np.float32)
    b = np.zeros(3, np.float32)
    lib().orc_frame(_f32(n), t, b)
    return t, b


def offset(p, n, tri):
    """p moved off the plane of triangle tri (3 vertices) along the unit n."""
    out = np.zeros(3, np.float32)
    lib().orc_offset(_f32(p), _f32(n), _f32(tri).reshape(-1), out)
    return out
