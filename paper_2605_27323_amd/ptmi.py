"""Python binding of libptmi (the C ABI in include/ptmi.h).

Argument marshalling only: every step of the path tracer runs in the HIP
library.  PyTorch provides device memory (tensors passed by pointer) and the
stream (torch.cuda.current_stream()).  Importing this module fails loudly if
the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PTMI_LIB") or os.path.join(HERE, "libptmi.so")

PT_OK, PT_EINVAL, PT_ENOMEM, PT_EHIP, PT_ESTATE, PT_EOVERFLOW, PT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MODE_MEGA, MODE_WAVE = 0, 1
FLAG_PROFILE, FLAG_NO_COMPACT, FLAG_SORT_MATERIAL, FLAG_COUNT_WORK, FLAG_SORT_RAYS = 1, 2, 4, 8, 16
FLAG_XCD_LOCAL = 32
FLAG_TWO_SLOT = 64
FLAG_KEEP_HITS = 128
FLAG_SERIAL_STAGES = 256
SAMPLER_PHILOX, SAMPLER_HALTON = 0, 1
STAGES = ["raygen", "extend", "shade", "shadow", "accumulate", "mega", "sort", "adjoint", "tail",
          "adjoint_radiance", "promote"]


class PtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ptmi error {code}: {msg}")
        self.code = code


class SceneDesc(C.Structure):
    _fields_ = [("nv", C.c_int32), ("nt", C.c_int32), ("nm", C.c_int32),
                ("positions", C.c_void_p), ("indices", C.c_void_p), ("tri_material", C.c_void_p),
                ("materials", C.c_void_p), ("albedo", C.c_void_p), ("emission", C.c_void_p),
                ("sky", C.c_float * 3)]


class BvhOpts(C.Structure):
    _fields_ = [("max_leaf", C.c_int32), ("threads", C.c_int32)]


class BvhInfo(C.Structure):
    _fields_ = [("node_count", C.c_int64), ("node_bytes", C.c_int64), ("tri_bytes", C.c_int64),
                ("light_count", C.c_int64), ("light_bytes", C.c_int64), ("material_bytes", C.c_int64),
                ("instance_count", C.c_int64), ("instance_bytes", C.c_int64), ("attribute_bytes", C.c_int64),
                ("depth", C.c_int32), ("stack_entries", C.c_int32), ("build_seconds", C.c_double)]


class InstancesDesc(C.Structure):
    _fields_ = [("n_meshes", C.c_int32), ("mesh_first", C.c_void_p), ("mesh_count", C.c_void_p),
                ("n_instances", C.c_int32), ("inst_mesh", C.c_void_p), ("o2w", C.c_void_p), ("w2o", C.c_void_p)]


class AttributesDesc(C.Structure):
    _fields_ = [("nv", C.c_int32), ("normals", C.c_void_p), ("uvs", C.c_void_p)]


class SceneBuffers(C.Structure):
    _fields_ = [("nodes", C.c_void_p), ("tris", C.c_void_p), ("lights", C.c_void_p), ("materials", C.c_void_p),
                ("albedo", C.c_void_p), ("emission", C.c_void_p), ("upload_params", C.c_int32),
                ("instances", C.c_void_p), ("attributes", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3),
                ("vfov_deg", C.c_double), ("width", C.c_int32), ("height", C.c_int32)]


class RenderArgs(C.Structure):
    _fields_ = [("spp", C.c_int32), ("max_depth", C.c_int32), ("seed", C.c_uint64), ("frame", C.c_uint32),
                ("job", C.c_uint32), ("nee", C.c_int32), ("rr_start", C.c_int32), ("mode", C.c_int32),
                ("flags", C.c_int32), ("block", C.c_int32), ("grid_mult", C.c_int32),
                ("sort_threshold", C.c_uint32), ("stack_lds", C.c_int32), ("tail_threshold", C.c_uint32),
                ("tail_bounce", C.c_int32), ("sampler", C.c_int32), ("tail_spread", C.c_int32),
                ("mega_waves", C.c_int32)]


NSTAGES = 11


class FrameStats(C.Structure):
    _fields_ = [("stage_ms", C.c_double * NSTAGES), ("launches", C.c_int64 * NSTAGES),
                ("stage_items", C.c_int64 * NSTAGES), ("stage_bytes", C.c_double * NSTAGES),
                ("node_visits", C.c_int64 * NSTAGES), ("tri_tests", C.c_int64 * NSTAGES),
                ("extension_rays", C.c_int64), ("shadow_rays", C.c_int64)]


class Job(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("args", RenderArgs), ("image_out", C.c_void_p)]


class BatchOpts(C.Structure):
    _fields_ = [("pool_capacity", C.c_uint32), ("block", C.c_int32), ("grid_mult", C.c_int32),
                ("stack_lds", C.c_int32), ("iters_per_graph", C.c_int32), ("use_graph", C.c_int32),
                ("pools", C.c_int32)]


class BatchResult(C.Structure):
    _fields_ = [("seconds", C.c_double), ("path_samples", C.c_int64), ("iterations", C.c_int64),
                ("launches", C.c_int64)]


# name -> (restype, argtypes); every function of include/ptmi.h
SIGNATURES = {
    "pt_version": (C.c_int32, []),
    "pt_last_error": (C.c_char_p, []),
    "pt_create": (C.c_int32, [C.POINTER(C.c_void_p), C.c_int32]),
    "pt_destroy": (C.c_int32, [C.c_void_p]),
    "pt_load_scene": (C.c_int32, [C.c_void_p, C.POINTER(SceneDesc)]),
    "pt_set_instances": (C.c_int32, [C.c_void_p, C.POINTER(InstancesDesc)]),
    "pt_set_attributes": (C.c_int32, [C.c_void_p, C.POINTER(AttributesDesc)]),
    "pt_build_bvh": (C.c_int32, [C.c_void_p, C.POINTER(BvhOpts), C.POINTER(BvhInfo)]),
    "pt_get_bvh": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "pt_bind_scene": (C.c_int32, [C.c_void_p, C.POINTER(SceneBuffers), C.c_void_p]),
    "pt_set_camera": (C.c_int32, [C.c_void_p, C.POINTER(Camera)]),
    "pt_workspace_size": (C.c_int32, [C.c_void_p, C.POINTER(RenderArgs), C.POINTER(C.c_uint64)]),
    "pt_render_frame": (C.c_int32, [C.c_void_p, C.POINTER(RenderArgs), C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_uint64, C.c_void_p]),
    "pt_render_frame_noalloc": (C.c_int32, [C.c_void_p, C.POINTER(RenderArgs), C.c_void_p, C.c_void_p, C.c_void_p]),
    "pt_frames_workspace_size": (C.c_int32, [C.c_void_p, C.POINTER(RenderArgs), C.POINTER(C.c_uint64)]),
    "pt_render_frames": (C.c_int32, [C.c_void_p, C.POINTER(RenderArgs), C.c_int32, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_uint64, C.c_void_p]),
    "pt_backward_workspace_size": (C.c_int32, [C.c_void_p, C.POINTER(RenderArgs), C.POINTER(C.c_uint64)]),
    "pt_render_backward": (C.c_int32, [C.c_void_p, C.POINTER(RenderArgs), C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_uint64, C.c_void_p]),
    "pt_frame_stats_get": (C.c_int32, [C.c_void_p, C.POINTER(FrameStats)]),
    "pt_batch_workspace_size": (C.c_int32, [C.POINTER(Job), C.c_int32, C.POINTER(BatchOpts), C.POINTER(C.c_uint64)]),
    "pt_render_batch": (C.c_int32, [C.POINTER(Job), C.c_int32, C.POINTER(BatchOpts), C.c_void_p, C.c_uint64, C.c_void_p,
                                    C.c_void_p, C.POINTER(BatchResult)]),
    "pt_sync": (C.c_int32, [C.c_void_p, C.c_void_p]),
}

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        # load torch's HIP runtime first: libptmi then binds to it (same
        # soname), so that one runtime serves torch's memory and our kernels
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_27323_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def check(code):
    if code != PT_OK:
        raise PtError(code, lib().pt_last_error().decode(errors="replace"))


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class Context:
    """A library context with a loaded scene and its built BVH (host side)."""

    def __init__(self, scene, device=0, max_leaf=0, threads=0, instances=None):
        """instances (optional): a two-level scene, dict of mesh_first,
        mesh_count (int32 [n_meshes]), inst_mesh (int32 [n_inst]), o2w and
        w2o (float32 [n_inst, 12], 3x4 row-major); the scene's triangles are
        then the meshes, in object space."""
        L = lib()
        h = C.c_void_p()
        check(L.pt_create(C.byref(h), int(device)))
        self.h = h
        self.device = device
        self._keep = []
        self.load(scene)
        if instances is not None:
            i = {k: _host(instances[k], np.int32) for k in ("mesh_first", "mesh_count", "inst_mesh")}
            i.update({k: _host(instances[k], np.float32) for k in ("o2w", "w2o")})
            d = InstancesDesc(i["mesh_first"].size, i["mesh_first"].ctypes.data, i["mesh_count"].ctypes.data,
                              i["inst_mesh"].size, i["inst_mesh"].ctypes.data, i["o2w"].ctypes.data,
                              i["w2o"].ctypes.data)
            check(L.pt_set_instances(self.h, C.byref(d)))
        opts = BvhOpts(max_leaf, threads)
        self.info = BvhInfo()
        check(L.pt_build_bvh(self.h, C.byref(opts), C.byref(self.info)))

    def load(self, scene):
        pos = _host(scene["positions"], np.float32)
        idx = _host(scene["indices"], np.int32)
        tm = _host(scene["tri_mat"], np.int32)
        mats = _host(scene["materials"], np.float32)
        alb = _host(scene["albedo"], np.float32)
        emi = _host(scene["emission"], np.float32)
        sky = np.asarray(scene["sky"], np.float32)
        self.nt = idx.size // 3
        d = SceneDesc(pos.size // 3, self.nt, mats.size // 4, pos.ctypes.data, idx.ctypes.data, tm.ctypes.data,
                      mats.ctypes.data, alb.ctypes.data, emi.ctypes.data, (C.c_float * 3)(*sky.tolist()))
        check(lib().pt_load_scene(self.h, C.byref(d)))
        nrm, uvs = scene.get("normals"), scene.get("uvs")
        if nrm is not None or uvs is not None:
            nrm = None if nrm is None else _host(nrm, np.float32)
            uvs = None if uvs is None else _host(uvs, np.float32)
            a = AttributesDesc(pos.size // 3, None if nrm is None else nrm.ctypes.data,
                               None if uvs is None else uvs.ctypes.data)
            check(lib().pt_set_attributes(self.h, C.byref(a)))
        self.albedo0 = alb.reshape(-1, 3)
        self.emission0 = emi.reshape(-1, 3)

    def host_bvh(self):
        """Host copies: nodes (uint8 [n,80]), tris (float32 [nt,12]), lights (uint32 [nl,4]:
        leaf-order index, CDF word, input index, 0)."""
        i = self.info
        nodes = np.zeros((i.node_count, 80), np.uint8)
        tris = np.zeros((max(self.nt, 1), 12), np.float32)
        lights = np.zeros((max(i.light_count, 1), 4), np.uint32)
        check(lib().pt_get_bvh(self.h, nodes.ctypes.data, tris.ctypes.data, lights.ctypes.data, None))
        return nodes, tris[:self.nt], lights[:i.light_count]

    def close(self):
        if getattr(self, "h", None):
            lib().pt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _aligned_empty(nbytes, device):
    import torch
    t = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t, t.data_ptr() + off


class Renderer(Context):
    """Scene bound to device buffers (torch tensors), plus a workspace."""

    def __init__(self, scene, camera=None, device=0, max_leaf=0, threads=0, instances=None):
        import torch
        super().__init__(scene, device=device, max_leaf=max_leaf, threads=threads, instances=instances)
        self.torch_device = torch.device("cuda", device)
        i = self.info
        self._bufs = {}
        ptrs = {}
        for name, nbytes in [("nodes", i.node_bytes), ("tris", i.tri_bytes), ("lights", i.light_bytes),
                             ("materials", i.material_bytes), ("instances", i.instance_bytes),
                             ("attributes", i.attribute_bytes)]:
            t, p = _aligned_empty(nbytes, self.torch_device)
            self._bufs[name] = t
            ptrs[name] = p
        self.albedo = torch.zeros((max(self.nt, 1), 3), dtype=torch.float32, device=self.torch_device)
        self.emission = torch.zeros((max(self.nt, 1), 3), dtype=torch.float32, device=self.torch_device)
        sb = SceneBuffers(ptrs["nodes"], ptrs["tris"], ptrs["lights"], ptrs["materials"],
                          self.albedo.data_ptr(), self.emission.data_ptr(), 1, ptrs["instances"],
                          ptrs["attributes"])
        check(lib().pt_bind_scene(self.h, C.byref(sb), self._stream()))
        self._ws = None
        self._ws_ptr = 0
        self._ws_bytes = 0
        if camera is not None:
            self.set_camera(camera)

    def _stream(self):
        import torch
        return C.c_void_p(torch.cuda.current_stream(self.torch_device).cuda_stream)

    def set_camera(self, cam):
        c = Camera((C.c_double * 3)(*cam["eye"]), (C.c_double * 3)(*cam["target"]), (C.c_double * 3)(*cam["up"]),
                   float(cam["vfov_deg"]), int(cam["width"]), int(cam["height"]))
        check(lib().pt_set_camera(self.h, C.byref(c)))
        self.width, self.height = int(cam["width"]), int(cam["height"])

    def args(self, spp=1, max_depth=5, seed=0, frame=0, job=0, nee=True, rr_start=-1, mode="wave", flags=0,
             block=0, grid_mult=0, sort_threshold=0, stack_lds=0, tail_threshold=0, tail_bounce=0,
             sampler="philox", tail_spread=False, mega_waves=0):
        m = MODE_WAVE if mode in ("wave", MODE_WAVE) else MODE_MEGA
        if sampler not in ("philox", "halton", SAMPLER_PHILOX, SAMPLER_HALTON):
            raise ValueError(f"unknown sampler {sampler!r} (philox or halton)")
        smp = SAMPLER_HALTON if sampler in ("halton", SAMPLER_HALTON) else SAMPLER_PHILOX
        return RenderArgs(int(spp), int(max_depth), int(seed), int(frame), int(job), int(bool(nee)), int(rr_start), m,
                          int(flags), int(block), int(grid_mult), int(sort_threshold), int(stack_lds),
                          int(tail_threshold), int(tail_bounce), smp, int(bool(tail_spread)), int(mega_waves))

    def workspace(self, a, backward=False):
        need = C.c_uint64()
        size = lib().pt_backward_workspace_size if backward else lib().pt_workspace_size
        check(size(self.h, C.byref(a), C.byref(need)))
        if need.value > self._ws_bytes:
            self._ws = None
            self._ws, self._ws_ptr = _aligned_empty(need.value, self.torch_device)
            self._ws_bytes = need.value
        return self._ws_ptr, self._ws_bytes

    def render(self, out=None, accum=None, **kw):
        """Render one frame; returns the (H, W, 3) float32 image tensor."""
        import torch
        a = self.args(**kw)
        if out is None:
            out = torch.empty((self.height, self.width, 3), dtype=torch.float32, device=self.torch_device)
        assert out.is_contiguous() and out.dtype == torch.float32 and out.numel() == self.height * self.width * 3
        ws, wsb = self.workspace(a)
        acc_ptr = None
        if accum is not None:
            assert accum.is_contiguous() and accum.numel() == out.numel()
            acc_ptr = accum.data_ptr()
        check(lib().pt_render_frame(self.h, C.byref(a), out.data_ptr(), acc_ptr, ws, wsb, self._stream()))
        return out

    def render_noalloc(self, out=None, accum=None, **kw):
        """Megakernel frame through pt_render_frame_noalloc (no workspace: the
        library's own per-GPU scratch); returns the image tensor."""
        import torch
        a = self.args(**dict(kw, mode="mega"))
        if out is None:
            out = torch.empty((self.height, self.width, 3), dtype=torch.float32, device=self.torch_device)
        assert out.is_contiguous() and out.dtype == torch.float32 and out.numel() == self.height * self.width * 3
        acc_ptr = None
        if accum is not None:
            assert accum.is_contiguous() and accum.numel() == out.numel()
            acc_ptr = accum.data_ptr()
        check(lib().pt_render_frame_noalloc(self.h, C.byref(a), out.data_ptr(), acc_ptr, self._stream()))
        return out

    def render_frames(self, n_frames, out=None, accum=None, **kw):
        """Render frames kw['frame'] .. + n_frames - 1 with frames in flight
        (pt_render_frames: three to eight, two less than the process's
        hardware queues); returns the image tensor (the last frame's image)."""
        import torch
        a = self.args(**kw)
        if out is None:
            out = torch.empty((self.height, self.width, 3), dtype=torch.float32, device=self.torch_device)
        assert out.is_contiguous() and out.dtype == torch.float32 and out.numel() == self.height * self.width * 3
        need = C.c_uint64()
        check(lib().pt_frames_workspace_size(self.h, C.byref(a), C.byref(need)))
        if need.value > getattr(self, "_fws_bytes", 0):
            self._fws = None
            self._fws, self._fws_ptr = _aligned_empty(need.value, self.torch_device)
            self._fws_bytes = need.value
        acc_ptr = None
        if accum is not None:
            assert accum.is_contiguous() and accum.numel() == out.numel()
            acc_ptr = accum.data_ptr()
        check(lib().pt_render_frames(self.h, C.byref(a), int(n_frames), out.data_ptr(), acc_ptr, self._fws_ptr,
                                     self._fws_bytes, self._stream()))
        return out

    def backward(self, d_image, d_albedo, d_emission, **kw):
        """Accumulate the adjoint into d_albedo / d_emission (nt x 3 tensors)."""
        a = self.args(**kw)
        ws, wsb = self.workspace(a, backward=True)
        d_image = d_image.contiguous()
        check(lib().pt_render_backward(self.h, C.byref(a), d_image.data_ptr(), d_albedo.data_ptr(),
                                       d_emission.data_ptr(), ws, wsb, self._stream()))

    def stats(self):
        s = FrameStats()
        check(lib().pt_frame_stats_get(self.h, C.byref(s)))
        return {"stage_ms": {STAGES[k]: s.stage_ms[k] for k in range(NSTAGES) if s.launches[k]},
                "launches": {STAGES[k]: s.launches[k] for k in range(NSTAGES) if s.launches[k]},
                "items": {STAGES[k]: s.stage_items[k] for k in range(NSTAGES) if s.stage_items[k]},
                "bytes": {STAGES[k]: s.stage_bytes[k] for k in range(NSTAGES) if s.stage_items[k]},
                "node_visits": {STAGES[k]: s.node_visits[k] for k in range(NSTAGES) if s.node_visits[k]},
                "tri_tests": {STAGES[k]: s.tri_tests[k] for k in range(NSTAGES) if s.tri_tests[k]},
                "extension_rays": s.extension_rays, "shadow_rays": s.shadow_rays}

    def sync(self):
        check(lib().pt_sync(self.h, self._stream()))


def _autograd():
    import torch

    class RenderFn(torch.autograd.Function):
        """image = render(albedo, emission): forward by the HIP renderer,
        backward by its path-replay adjoint (same seed/frame/spp, so the
        gradient is that of the fixed-sample estimator)."""

        @staticmethod
        def forward(ctx, albedo, emission, renderer, kw):
            if albedo.data_ptr() != renderer.albedo.data_ptr():
                renderer.albedo.copy_(albedo.detach())
            if emission.data_ptr() != renderer.emission.data_ptr():
                renderer.emission.copy_(emission.detach())
            ctx.renderer = renderer
            ctx.kw = dict(kw)
            return renderer.render(**kw).clone()

        @staticmethod
        def backward(ctx, grad_image):
            R = ctx.renderer
            ga = torch.zeros_like(R.albedo)
            ge = torch.zeros_like(R.emission)
            kw = {k: v for k, v in ctx.kw.items() if k != "mode"}
            R.backward(grad_image.contiguous(), ga, ge, **kw)
            return ga, ge, None, None

    return RenderFn


_RENDER_FN = None


def render_differentiable(albedo, emission, renderer, **kw):
    """Differentiable render: gradients flow to albedo and emission (nt x 3)."""
    global _RENDER_FN
    if _RENDER_FN is None:
        _RENDER_FN = _autograd()
    return _RENDER_FN.apply(albedo, emission, renderer, kw)


def render_batch(renderers, job_args, images=None, pool_capacity=0, block=0, grid_mult=0, iters_per_graph=0,
                 use_graph=True, workspace=None, stack_lds=0, pools=0):
    """Render several jobs in one batched persistent wavefront.

    renderers: Renderer per job (scene bound, camera set, all on one device);
    job_args: dict of render arguments per job (spp, max_depth, seed, frame,
    nee, rr_start; `job` defaults to the job's index); pools: pools run
    concurrently (0 = 1).  Returns (images, per-job completion ms, result
    dict)."""
    import torch
    n = len(renderers)
    jobs = (Job * n)()
    if images is None:
        images = [torch.empty((R.height, R.width, 3), dtype=torch.float32, device=R.torch_device) for R in renderers]
    for j, (R, kw) in enumerate(zip(renderers, job_args)):
        kw = dict(kw)
        kw.setdefault("job", j)
        jobs[j].ctx = R.h
        jobs[j].args = R.args(**kw)
        jobs[j].image_out = images[j].data_ptr()
    opts = BatchOpts(int(pool_capacity), int(block), int(grid_mult), int(stack_lds), int(iters_per_graph),
                     int(bool(use_graph)), int(pools))
    need = C.c_uint64()
    check(lib().pt_batch_workspace_size(jobs, n, C.byref(opts), C.byref(need)))
    if workspace is None or workspace[1] < need.value:
        t, p = _aligned_empty(need.value, renderers[0].torch_device)
        workspace = (t, need.value, p)
    ms = np.zeros(n, np.float64)
    res = BatchResult()
    stream = renderers[0]._stream()
    check(lib().pt_render_batch(jobs, n, C.byref(opts), workspace[2], workspace[1], stream, ms.ctypes.data,
                                C.byref(res)))
    out = {"seconds": res.seconds, "path_samples": res.path_samples, "iterations": res.iterations,
           "launches": res.launches, "workspace": workspace}
    return images, ms, out
