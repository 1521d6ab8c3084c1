"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import numpy as np

import oracle


def image_tolerance_report(gpu, ref, fragile):
    """Per-pixel check: all channels |g - o| <= 1e-4 max(|g|, |o|) + 1e-6 mean(o).

    Returns (pass_fraction, n_fail, n_unexplained, n_bit_exact)."""
    g = np.asarray(gpu, np.float64).reshape(-1, 3)
    o = np.asarray(ref, np.float64).reshape(-1, 3)
    tol = 1e-4 * np.maximum(np.abs(g), np.abs(o)) + 1e-6 * max(float(o.mean()), 1e-30)
    ok = (np.abs(g - o) <= tol).all(1)
    fr = np.asarray(fragile).reshape(-1) != 0
    exact = (np.asarray(gpu, np.float32).reshape(-1, 3).view(np.uint32) ==
             np.asarray(ref, np.float32).reshape(-1, 3).view(np.uint32)).all(1)
    return ok.mean(), int((~ok).sum()), int((~ok & ~fr).sum()), int(exact.sum())


def assert_parity(gpu, ref, fragile, min_pass=0.999, what=""):
    frac, nfail, unexplained, nexact = image_tolerance_report(gpu, ref, fragile)
    n = np.asarray(ref).reshape(-1, 3).shape[0]
    msg = f"{what}: pass {frac:.6f} ({nfail} fail, {unexplained} unexplained), bit-exact {nexact}/{n}"
    print(msg, flush=True)
    assert frac >= min_pass, msg
    assert unexplained == 0, msg
    return nexact


def oracle_image(scene, cam, pixels=None, **kw):
    S = oracle.Scene(scene)
    img, frag = S.render(cam, pixels=pixels, **kw)
    return img, frag, S


def degenerate_scene(only_degenerate_lights=False):
    """The Cornell box (24 x 20) plus three zero-area triangles: collinear
    vertices, a repeated vertex (emissive) and a single point (emissive).
    With only_degenerate_lights the box's own light is switched off, so
    every emitter has zero area and the sky is the only light."""
    from paper_2605_27323_amd import scenes
    scene, cam = scenes.cornell()
    cam = dict(cam, width=24, height=20)
    s = {k: v.copy() for k, v in scene.items()}
    nv = s["positions"].shape[0]
    extra_p = np.array([[0.2, 0.2, 0.2], [0.3, 0.3, 0.3], [0.4, 0.4, 0.4], [0.1, 0.5, 0.3]], np.float32)
    s["positions"] = np.concatenate([s["positions"], extra_p])
    s["indices"] = np.concatenate([s["indices"], np.array([[nv, nv + 1, nv + 2], [nv + 3, nv + 3, nv],
                                                           [nv, nv, nv]], np.int32)])
    s["tri_mat"] = np.concatenate([s["tri_mat"], np.zeros(3, np.int32)])
    s["albedo"] = np.concatenate([s["albedo"], np.full((3, 3), 0.5, np.float32)])
    s["emission"] = np.concatenate([s["emission"], np.array([[0, 0, 0], [5, 5, 5], [3, 3, 3]], np.float32)])
    if only_degenerate_lights:
        s["emission"][:-3] = 0.0
        s["sky"] = np.array([0.3, 0.3, 0.3], np.float32)
    return s, cam
