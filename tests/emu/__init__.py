"""CPU emulator of the HIP kernels (tests only): builds libptmi_emu.so from
the library sources plus emu.hip, compiled for the host."""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
LIB = os.path.join(HERE, "libptmi_emu.so")
_L = None


def build():
    from paper_2605_27323_amd import build as B
    csrc = os.path.join(ROOT, "paper_2605_27323_amd", "csrc")
    srcs = [os.path.join(HERE, "emu.hip"), os.path.join(csrc, "kernels.hip"), os.path.join(csrc, "bvh_build.cpp")]
    for extra in ("adjoint.hip", "batch.hip", "noalloc.hip"):
        p = os.path.join(csrc, extra)
        if os.path.exists(p):
            srcs.append(p)
    cmd = [B.HIPCC, *B.COMMON, "-shared", "-x", "hip", *srcs, "-o", LIB + ".tmp", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)


def _stale():
    """True when the emulator library is missing or older than a source."""
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    if os.path.getmtime(os.path.abspath(__file__)) > t:
        return True
    dirs = [HERE, os.path.join(ROOT, "paper_2605_27323_amd", "csrc"), os.path.join(ROOT, "include")]
    for d in dirs:
        for f in os.listdir(d):
            if f.endswith((".h", ".hip", ".cpp")) and os.path.getmtime(os.path.join(d, f)) > t:
                return True
    return False


def lib():
    global _L
    if _L is None:
        from paper_2605_27323_amd import ptmi
        ptmi.lib()  # torch's HIP runtime first
        if _stale():
            build()
        L = C.CDLL(LIB)
        L.emu_render_mega.restype = C.c_int32
        L.emu_render_mega.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                      C.c_uint32, C.c_uint32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]
        L.emu_render_wave.restype = C.c_int32
        L.emu_render_wave.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32,
                                      C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.c_int32, C.c_uint32, C.c_void_p,
                                      C.c_void_p, C.c_int32]
        L.emu_closest.restype = C.c_int32
        L.emu_closest.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p]
        L.emu_render_batch.restype = C.c_int64
        L.emu_render_batch.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64, C.c_void_p]
        L.emu_backward.restype = C.c_int32
        L.emu_backward.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int32,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]
        for name, (res, args) in ptmi.SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _L = L
    return _L


class Emu:
    """Host-only library context (emulator build) with a scene and camera."""

    def __init__(self, scene, cam, max_leaf=0, instances=None):
        from paper_2605_27323_amd import ptmi
        L = lib()
        h = C.c_void_p()
        assert L.pt_create(C.byref(h), -1) == 0
        self.h = h
        keep = {k: np.ascontiguousarray(v) for k, v in scene.items()}
        for k in ("normals", "uvs"):
            if k in keep:
                keep[k] = np.ascontiguousarray(keep[k], np.float32)
        self._keep = keep
        d = ptmi.SceneDesc(keep["positions"].shape[0], keep["indices"].shape[0], keep["materials"].shape[0],
                           keep["positions"].ctypes.data, keep["indices"].ctypes.data, keep["tri_mat"].ctypes.data,
                           keep["materials"].ctypes.data, keep["albedo"].ctypes.data, keep["emission"].ctypes.data,
                           (C.c_float * 3)(*np.asarray(keep["sky"], np.float32).tolist()))
        assert L.pt_load_scene(h, C.byref(d)) == 0, L.pt_last_error()
        if "normals" in keep or "uvs" in keep:
            a = ptmi.AttributesDesc(keep["positions"].shape[0],
                                    keep["normals"].ctypes.data if "normals" in keep else None,
                                    keep["uvs"].ctypes.data if "uvs" in keep else None)
            assert L.pt_set_attributes(h, C.byref(a)) == 0, L.pt_last_error()
        if instances is not None:
            ik = {k: np.ascontiguousarray(instances[k], np.int32) for k in ("mesh_first", "mesh_count", "inst_mesh")}
            ik.update({k: np.ascontiguousarray(instances[k], np.float32) for k in ("o2w", "w2o")})
            self._keep_inst = ik
            idesc = ptmi.InstancesDesc(ik["mesh_first"].size, ik["mesh_first"].ctypes.data, ik["mesh_count"].ctypes.data,
                                       ik["inst_mesh"].size, ik["inst_mesh"].ctypes.data, ik["o2w"].ctypes.data,
                                       ik["w2o"].ctypes.data)
            assert L.pt_set_instances(h, C.byref(idesc)) == 0, L.pt_last_error()
        info = ptmi.BvhInfo()
        opts = ptmi.BvhOpts(int(max_leaf), 0)
        assert L.pt_build_bvh(h, C.byref(opts), C.byref(info)) == 0
        c = ptmi.Camera((C.c_double * 3)(*cam["eye"]), (C.c_double * 3)(*cam["target"]), (C.c_double * 3)(*cam["up"]),
                        float(cam["vfov_deg"]), int(cam["width"]), int(cam["height"]))
        assert L.pt_set_camera(h, C.byref(c)) == 0
        self.W, self.H = int(cam["width"]), int(cam["height"])

    def closest(self, o, d):
        """Closest hit of the library's traversal: t, input id (-1 on a miss), b1, b2."""
        o = np.ascontiguousarray(o, np.float32).reshape(-1, 3)
        d = np.ascontiguousarray(d, np.float32).reshape(-1, 3)
        n = o.shape[0]
        t = np.zeros(n, np.float32)
        i = np.zeros(n, np.int32)
        b1 = np.zeros(n, np.float32)
        b2 = np.zeros(n, np.float32)
        assert lib().emu_closest(self.h, n, o.ctypes.data, d.ctypes.data, t.ctypes.data, i.ctypes.data,
                                 b1.ctypes.data, b2.ctypes.data) == 0
        return t, i, b1, b2

    def mega(self, pixels=None, spp=1, max_depth=5, seed=0, frame=0, job=0, nee=True, rr_start=-1, sampler=0):
        if pixels is None:
            pixels = np.arange(self.W * self.H, dtype=np.int32)
        pixels = np.ascontiguousarray(pixels, np.int32)
        out = np.zeros((pixels.size, 3), np.float32)
        rays = np.zeros(2, np.uint64)
        rc = lib().emu_render_mega(self.h, pixels.ctypes.data, pixels.size, spp, max_depth, seed, frame, job,
                                   int(bool(nee)), rr_start, out.ctypes.data, rays.ctypes.data, int(sampler))
        assert rc == 0
        return out, rays

    def wave(self, spp=1, max_depth=5, seed=0, frame=0, job=0, nee=True, rr_start=-1, compact=True, shuffle=0,
             sort=False, tail=0, sampler=0):
        img = np.zeros((self.W * self.H, 3), np.float32)
        rays = np.zeros(2, np.uint64)
        rc = lib().emu_render_wave(self.h, spp, max_depth, seed, frame, job, int(bool(nee)), rr_start,
                                   int(bool(compact)), shuffle, int(bool(sort)), int(tail), img.ctypes.data,
                                   rays.ctypes.data, int(sampler))
        assert rc == 0
        return img, rays

    def backward(self, d_image, spp=1, max_depth=5, seed=0, frame=0, job=0, nee=True, sampler=0, keep_hits=False):
        d_image = np.ascontiguousarray(d_image, np.float32).reshape(-1, 3)
        nt = self._keep["indices"].shape[0]
        ga = np.zeros((max(nt, 1), 3), np.float32)
        ge = np.zeros((max(nt, 1), 3), np.float32)
        rc = lib().emu_backward(self.h, spp, max_depth, seed, frame, job, int(bool(nee)), d_image.ctypes.data,
                                ga.ctypes.data, ge.ctypes.data, int(sampler), int(keep_hits))
        assert rc == 0
        return ga[:nt], ge[:nt]

    def __del__(self):
        try:
            lib().pt_destroy(self.h)
        except Exception:
            pass


def render_batch(emus, job_args, capacity, shuffle=0):
    """Emulated batched pool; returns (list of images, iterations)."""
    from paper_2605_27323_amd import ptmi
    n = len(emus)
    ctxs = (C.c_void_p * n)(*[e.h.value for e in emus])
    args = (ptmi.RenderArgs * n)()
    total_pix = 0
    for j, (e, kw) in enumerate(zip(emus, job_args)):
        a = dict(spp=1, max_depth=5, seed=0, frame=0, job=j, nee=True, rr_start=-1, sampler=0)
        a.update(kw)
        args[j] = ptmi.RenderArgs(a["spp"], a["max_depth"], a["seed"], a["frame"], a["job"], int(bool(a["nee"])),
                                  a["rr_start"], 1, 0, 0, 0, 0, sampler=int(a["sampler"]))
        total_pix += e.W * e.H
    img = np.zeros((total_pix, 3), np.float32)
    it = lib().emu_render_batch(ctxs, args, n, capacity, shuffle, img.ctypes.data)
    assert it >= 0, "batch bookkeeping error"
    out, off = [], 0
    for e in emus:
        out.append(img[off:off + e.W * e.H])
        off += e.W * e.H
    return out, it
