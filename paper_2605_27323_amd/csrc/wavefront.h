// Per-item bodies of the wavefront stages (paper Sec. 2.3 and 3.1), shared
// by the HIP kernels and the CPU emulator used in tests.  The kernels add
// only the grid-stride loops and the wave-level queue compaction.
#pragma once
#include "kernels.h"

namespace ptmi {

PT_DEV void store_pixel(float* __restrict__ img, float* __restrict__ acc, uint32_t pix, f3 I, uint32_t frame) {
    img[3 * (size_t)pix + 0] = I.x;
    img[3 * (size_t)pix + 1] = I.y;
    img[3 * (size_t)pix + 2] = I.z;
    if (acc) {
        float* a = acc + 3 * (size_t)pix;
        if (frame == 0) {
            a[0] = I.x;
            a[1] = I.y;
            a[2] = I.z;
        } else {
            float n = (float)(frame + 1u);
            a[0] = a[0] + (I.x - a[0]) / n;
            a[1] = a[1] + (I.y - a[1]) / n;
            a[2] = a[2] + (I.z - a[2]) / n;
        }
    }
}

// camera ray and initial state of path p = pixel * spp + s (queue 0 slot p)
PT_DEV void raygen_item(const CamView& cam, const PathParams& pp, const WaveBufs& wb, uint32_t p) {
    const uint32_t pix = p / (uint32_t)pp.spp;
    const uint32_t s = p - pix * (uint32_t)pp.spp;
    const uint32_t sample = pp.frame * (uint32_t)pp.spp + s;
    f3 o, d;
    camera_sample(cam, pp, pix, sample, o, d);
    wb.ray_o[0][p] = make_float4(o.x, o.y, o.z, u2f(p));
    wb.ray_d[0][p] = make_float4(d.x, d.y, d.z, 0.f);
    wb.pst[0][p] = make_float4(1.f, 1.f, 1.f, u2f(0u));
    wb.L[p] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// closest hit of queue slot i of bounce b: the hit record is (t, instance
// record in a two-level scene, 0, leaf-order triangle)
template <int LDS, bool COUNT = false, bool INST = false>
PT_DEV void extend_item(const SceneView& sc, const WaveBufs& wb, int b, uint32_t i, TravStack<LDS, COUNT>& st) {
    float4 o4 = wb.ray_o[b & 1][i], d4 = wb.ray_d[b & 1][i];
    if (f2u(o4.w) == kDeadPath) return;
    Hit h = closest_hit_t<LDS, COUNT, INST>(sc, xyz(o4), xyz(d4), INFINITY, st);
    wb.hit[i] = make_float4(h.t, INST ? u2f(h.inst) : 0.f, 0.f, u2f(h.tri));
}

// 6-bit sort key of a hit: material type in bits 4-5, low bits of the
// material index in bits 0-3; 63 for a miss
PT_DEV uint32_t material_key(const SceneView& sc, const float4& h4) {
    const uint32_t tri = f2u(h4.w);
    if (tri >= (uint32_t)sc.nt) return 63u;
    const uint32_t mi = f2u(sc.tris[(size_t)tri * 3 + 1].w) & ~kLightFlag;
    const uint32_t type = (uint32_t)sc.mats[mi].x;
    return (type << 4) | (mi & 15u);
}

// 6-bit sort key of a queued ray: direction octant in bits 3-5, the side of
// the scene centre the origin lies on per axis in bits 0-2; rays with equal
// keys tend to visit the same BVH nodes
PT_DEV uint32_t ray_key(const SceneView& sc, const float4& o4, const float4& d4) {
    return ((d4.x < 0.0f) ? 32u : 0u) | ((d4.y < 0.0f) ? 16u : 0u) | ((d4.z < 0.0f) ? 8u : 0u) |
           ((o4.x > sc.cx) ? 4u : 0u) | ((o4.y > sc.cy) ? 2u : 0u) | ((o4.z > sc.cz) ? 1u : 0u);
}

// shade queue slot i of bounce b (vertex k = b + 1); returns the path id
// (kDeadPath for a dead slot); vo / sh / ps describe what to enqueue.  With
// a material sort the slot's data is read from slot perm[i].  The path
// radiance L[path] is read only where this vertex adds to it, and updated
// in place; with for_tail it is always read into ps.L (plus this vertex's
// term) for finish_path, which stores it at the path's end.
template <bool INST = false, bool ATTR = false>
PT_DEV uint32_t shade_item(const SceneView& sc, const PathParams& pp, const WaveBufs& wb, int b, uint32_t i,
                           VertexOut& vo, ShadowReq& sh, PathState& ps, const uint32_t* __restrict__ perm = nullptr,
                           const LightCache& lc = no_light_cache(), bool for_tail = false) {
    if (perm) i = perm[i];
    const int cur = b & 1;
    // all four records at once (a dead slot's stale records are not used);
    // the empty asm consumes them before the dead-slot test so that the
    // compiler cannot sink three of the loads behind it
    const float4 o4 = wb.ray_o[cur][i], d4 = wb.ray_d[cur][i], p4 = wb.pst[cur][i], h4 = wb.hit[i];
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" ::"v"(d4.x), "v"(p4.x), "v"(h4.w));
#endif
    const uint32_t path = f2u(o4.w);
    vo.cont = false;
    sh.valid = false;
    if (path == kDeadPath) return path;
    const uint32_t pix = path / (uint32_t)pp.spp;
    const uint32_t s = path - pix * (uint32_t)pp.spp;
    const uint32_t sample = pp.frame * (uint32_t)pp.spp + s;
    ps.beta = xyz(p4);
    ps.L = mk3(0.f, 0.f, 0.f);
    ps.p_prev = d4.w;
    ps.prev_smooth = (int)f2u(p4.w);
    Hit h;
    h.t = h4.x;
    h.tri = f2u(h4.w);
    h.id = 0;
    if constexpr (INST) {
        h.inst = f2u(h4.y);
        hit_barycentrics_inst(sc, xyz(o4), xyz(d4), h);
    } else {
        hit_barycentrics(sc, xyz(o4), xyz(d4), h);
    }
    if (wb.rec_hit) wb.rec_hit[(size_t)b * wb.rec_n + path] = make_uint2(f2u(h.t), h.tri);
    vo = shade_vertex<INST, ATTR>(sc, pp, pix, sample, b + 1, xyz(d4), h, ps, sh, lc);
    if (for_tail) {
        ps.L = xyz(wb.L[path]);
        add_radiance(ps, vo);
    } else if (vo.addL) {
        ps.L = xyz(wb.L[path]);
        add_radiance(ps, vo);
        wb.L[path] = make_float4(ps.L.x, ps.L.y, ps.L.z, 0.f);
    }
    return path;
}

// Hybrid tail: continue a shaded path in place to its end (megakernel
// order: light sample of the current vertex, then extend and shade the next
// vertices) and store its final radiance.  Used when a bounce's queue is too
// short to keep the wavefront stages busy.
// n_ext / n_sh count the extension and shadow rays traced here.
template <int LDS, bool COUNT = false, bool INST = false, bool ATTR = false>
PT_DEV void finish_path(const SceneView& sc, const PathParams& pp, const WaveBufs& wb, uint32_t path, int k,
                        VertexOut vo, ShadowReq sh, PathState& ps, TravStack<LDS, COUNT>& st, uint32_t& n_ext,
                        uint32_t& n_sh, const LightCache& lc = no_light_cache()) {
    const uint32_t pix = path / (uint32_t)pp.spp;
    const uint32_t s = path - pix * (uint32_t)pp.spp;
    const uint32_t sample = pp.frame * (uint32_t)pp.spp + s;
    while (true) {
        if (sh.valid) {
            ++n_sh;
            const bool seen = !any_hit_t<LDS, COUNT, INST>(sc, sh.o, sh.d, kShadowTmax, st);
            if (seen) ps.L = mk3(ps.L.x + sh.contrib.x, ps.L.y + sh.contrib.y, ps.L.z + sh.contrib.z);
            if (wb.rec_vis) wb.rec_vis[(size_t)(k - 1) * wb.rec_n + path] = seen ? 1 : 0;
        }
        if (!vo.cont) break;
        ++k;
        ++n_ext;
        const f3 d = vo.d;
        Hit h = closest_hit_t<LDS, COUNT, INST>(sc, vo.o, d, INFINITY, st);
        if (wb.rec_hit) wb.rec_hit[(size_t)(k - 1) * wb.rec_n + path] = make_uint2(f2u(h.t), h.tri);
        vo = shade_vertex<INST, ATTR>(sc, pp, pix, sample, k, d, h, ps, sh, lc);
        add_radiance(ps, vo);
    }
    wb.L[path] = make_float4(ps.L.x, ps.L.y, ps.L.z, 0.f);
}

PT_DEV void write_continuation(const WaveBufs& wb, int nxt, uint32_t j, const VertexOut& vo, const PathState& ps,
                               uint32_t path) {
    wb.ray_o[nxt][j] = make_float4(vo.o.x, vo.o.y, vo.o.z, u2f(path));
    wb.ray_d[nxt][j] = make_float4(vo.d.x, vo.d.y, vo.d.z, ps.p_prev);
    wb.pst[nxt][j] = make_float4(ps.beta.x, ps.beta.y, ps.beta.z, u2f((uint32_t)ps.prev_smooth));
}

PT_DEV void write_dead(const WaveBufs& wb, int nxt, uint32_t j) {
    wb.ray_o[nxt][j] = make_float4(0.f, 0.f, 0.f, u2f(kDeadPath));
}

PT_DEV void write_shadow(const WaveBufs& wb, uint32_t j, const ShadowReq& sh, uint32_t path) {
    wb.sh_o[j] = make_float4(sh.o.x, sh.o.y, sh.o.z, u2f(path));
    wb.sh_d[j] = make_float4(sh.d.x, sh.d.y, sh.d.z, 0.f);
    wb.sh_c[j] = make_float4(sh.contrib.x, sh.contrib.y, sh.contrib.z, 0.f);
}

// unoccluded light-sample segment i: add its beta * C to its path
PT_DEV void shadow_add(const WaveBufs& wb, uint32_t i) {
    const uint32_t path = f2u(wb.sh_o[i].w);
    float4 c4 = wb.sh_c[i];
    float4 l4 = wb.L[path];
    wb.L[path] = make_float4(l4.x + c4.x, l4.y + c4.y, l4.z + c4.z, 0.f);
}

// the visibility of light-sample segment i of bounce b, for the adjoint's
// kept records
PT_DEV void shadow_record(const WaveBufs& wb, int b, uint32_t i, bool seen) {
    if (wb.rec_vis) wb.rec_vis[(size_t)b * wb.rec_n + f2u(wb.sh_o[i].w)] = seen ? 1 : 0;
}

// light-sample segment i of bounce b: add beta * C to its path when
// unoccluded
template <int LDS, bool COUNT = false, bool INST = false>
PT_DEV void shadow_item(const SceneView& sc, const WaveBufs& wb, int b, uint32_t i, TravStack<LDS, COUNT>& st) {
    float4 o4 = wb.sh_o[i], d4 = wb.sh_d[i];
    const bool seen = !any_hit_t<LDS, COUNT, INST>(sc, xyz(o4), xyz(d4), kShadowTmax, st);
    if (seen) shadow_add(wb, i);
    shadow_record(wb, b, i, seen);
}

// per-pixel mean over its spp paths, summed in sample order
PT_DEV void accumulate_item(const PathParams& pp, const float4* __restrict__ L, float* __restrict__ img,
                            float* __restrict__ acc, uint32_t pix) {
    const float4* l = L + (size_t)pix * (uint32_t)pp.spp;
    f3 sum = xyz(l[0]);
    for (int s = 1; s < pp.spp; ++s) sum = add3(sum, xyz(l[s]));
    const float fs = (float)pp.spp;
    store_pixel(img, acc, pix, mk3(sum.x / fs, sum.y / fs, sum.z / fs), pp.frame);
}

}  // namespace ptmi
