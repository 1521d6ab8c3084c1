// Path-replay adjoint of one camera path (Vicini, Speierer, Jakob, "Path
// Replay Backpropagation", SIGGRAPH 2021), shared by the HIP kernel and the
// CPU emulator.  With sampling independent of albedo and emission (cosine
// and visible-normal sampling, area-proportional light picks, no roulette)
// the path is fixed by its random numbers, so it is replayed twice instead
// of being stored: replay A recomputes the radiance L of the path, replay B
// walks it again and, at each vertex x_k with throughput beta_k,
//   emission w Le(tri_k):      dLe(tri_k)   += delta beta_k w
//   light sample f Le(y) G:    dLe(tri_y)   += delta beta_k f G
//                              dalb(tri_k)  += delta beta_k df/dalb G Le(y)
//   continuation weight W_k:   dalb(tri_k)  += delta (L - L_acc) dW/dalb / W
// where L_acc is the radiance gathered up to and including x_k's light
// sample and delta = dLoss/dI(pixel) / spp.  Channels with W = 0 carry no
// gradient through W (the division of the method).  The accumulator takes
// add_tri(hot, which, c, p, v) for channel c of the albedo (which = 0) or
// emission (1) of the hit triangle, at p, hot being its slot among the
// largest triangles + 1 (0 = none), and add_light(j, c, p, v) for the
// emission of light j of the light table; both skip v = 0.
#pragma once
#include "device.h"

namespace ptmi {

// Intersections kept by replay A (optional): for vertex k (1-based) of path
// p, at [(k - 1) * npaths + p], the hit of the ray that reached it (t, the
// triangle's leaf-order index, ~0u for a miss) and whether its light
// sample was traced and unoccluded (1) or not (0).  Replay B then reads
// them instead of tracing the same rays again: the intersection is a pure
// function of the ray and the scene, so the replay is the same.
struct VertexRecs {
    uint2* __restrict__ hit;
    uint8_t* __restrict__ vis;
    uint32_t npaths;
};

// One vertex of replay A that keeps its records: path_vertex of the
// megakernel plus the two stores (the same radiance bit for bit).
template <int LDS, bool ATTR = false, bool COUNT = false>
PT_DEV bool adjoint_a_vertex(const SceneView& sc, const PathParams& pp, uint32_t pix, uint32_t sample, uint32_t path,
                             PathRun& pr, TravStack<LDS, COUNT>& st, uint32_t& n_ext, uint32_t& n_sh,
                             const VertexRecs& rec) {
    Hit h = closest_hit<LDS>(sc, make_ray(pr.o, pr.d), INFINITY, st);
    ++n_ext;
    const size_t at = (size_t)(pr.k - 1) * rec.npaths + path;
    rec.hit[at] = make_uint2(f2u(h.t), h.tri);
    ShadowReq sh;
    VertexOut vo = shade_vertex<false, ATTR>(sc, pp, pix, sample, pr.k, pr.d, h, pr.ps, sh);
    add_radiance(pr.ps, vo);
    uint8_t seen = 0;
    if (sh.valid) {
        ++n_sh;
        if (!any_hit<LDS>(sc, make_ray(sh.o, sh.d), kShadowTmax, st)) {
            pr.ps.L = mk3(pr.ps.L.x + sh.contrib.x, pr.ps.L.y + sh.contrib.y, pr.ps.L.z + sh.contrib.z);
            seen = 1;
        }
    }
    rec.vis[at] = seen;
    if (!vo.cont) return false;
    pr.o = vo.o;
    pr.d = vo.d;
    ++pr.k;
    return true;
}

// Replay B of one path as resumable steps, one path vertex per step, from
// the path's radiance Ltot (replay A), so that a kernel can hand a lane
// whose path has ended the next path while the others go on.
struct AdjRun {
    PathRun pr;  // ray, throughput and radiance gathered so far
    f3 Ltot;     // radiance of the whole path
    f3 delta;    // dLoss/dI(pixel) / spp
    uint32_t pix, sample;
    uint32_t path;  // index of the path sample (its records with STORED)
};

PT_DEV void adjoint_b_begin(const CamView& cam, const PathParams& pp, uint32_t pix, uint32_t sample, f3 delta,
                            f3 Ltot, AdjRun& ar, uint32_t path = 0) {
    path_begin(cam, pp, pix, sample, ar.pr);
    ar.Ltot = Ltot;
    ar.delta = delta;
    ar.pix = pix;
    ar.sample = sample;
    ar.path = path;
}

// One vertex of replay B; returns false when the path is finished.  ATTR:
// the scene may have vertex attributes (see shade_vertex).  STORED: the
// vertex's intersection and light-sample visibility come from replay A's
// records (rec) and no ray is traced.  The vertex's extension and shadow
// rays (traced here, or by replay A with STORED) are counted in n_ext, n_sh.
template <int LDS, bool ATTR = false, class Acc, bool COUNT = false, bool STORED = false>
PT_DEV bool adjoint_b_step(const SceneView& sc, const PathParams& pp, AdjRun& ar, float* __restrict__ g_alb,
                           float* __restrict__ g_emi, TravStack<LDS, COUNT>& st, Acc& acc, uint32_t& n_ext,
                           uint32_t& n_sh, const VertexRecs& rec = VertexRecs{nullptr, nullptr, 0u}) {
    const f3 delta = ar.delta, Ltot = ar.Ltot;
    const uint32_t pix = ar.pix, sample = ar.sample;
    const int k = ar.pr.k;
    const f3 o = ar.pr.o, d = ar.pr.d;
    PathState& ps = ar.pr.ps;
    size_t at = 0;
    Hit h;
    if constexpr (STORED) {
        at = (size_t)(k - 1) * rec.npaths + ar.path;
        const uint2 r = rec.hit[at];
        h.t = u2f(r.x);
        h.tri = r.y;
        h.id = 0;
        hit_barycentrics(sc, o, d, h);
    } else {
        Ray ray = make_ray(o, d);
        h = closest_hit<LDS>(sc, ray, INFINITY, st);
    }
    ++n_ext;
    const f3 beta = ps.beta;
    ShadowReq sh;
    VertexOut vo = shade_vertex<false, ATTR>(sc, pp, pix, sample, k, d, h, ps, sh);
    add_radiance(ps, vo);
    if (vo.id == 0xFFFFFFFFu) return false;  // escaped: the sky is not a parameter
    const uint32_t id = vo.id;
    if (vo.emitted) {
        acc.add_tri(vo.hot, 1, 0, g_emi + 3 * (size_t)id + 0, delta.x * (beta.x * vo.w_emit));
        acc.add_tri(vo.hot, 1, 1, g_emi + 3 * (size_t)id + 1, delta.y * (beta.y * vo.w_emit));
        acc.add_tri(vo.hot, 1, 2, g_emi + 3 * (size_t)id + 2, delta.z * (beta.z * vo.w_emit));
    }
    // the albedo gradient of this vertex: light-sample and continuation
    // terms summed here, one accumulation per channel
    float ga[3] = {0.0f, 0.0f, 0.0f};
    if (sh.valid) {
        bool seen;
        ++n_sh;
        if constexpr (STORED) seen = rec.vis[at] != 0;
        else seen = !any_hit<LDS>(sc, make_ray(sh.o, sh.d), kShadowTmax, st);
        if (seen) {
            ps.L = mk3(ps.L.x + sh.contrib.x, ps.L.y + sh.contrib.y, ps.L.z + sh.contrib.z);
            const f3 rho = load3(sc.albedo, id);
            const f3 Le = load3(sc.emission, sh.light_id);
            const float der = lobe_der(sh.lobe);
            const uint32_t lid = sh.light_id;
            acc.add_light(sh.light_idx, 0, g_emi + 3 * (size_t)lid + 0,
                          delta.x * (beta.x * (lobe_value(sh.lobe, rho.x) * sh.G)));
            acc.add_light(sh.light_idx, 1, g_emi + 3 * (size_t)lid + 1,
                          delta.y * (beta.y * (lobe_value(sh.lobe, rho.y) * sh.G)));
            acc.add_light(sh.light_idx, 2, g_emi + 3 * (size_t)lid + 2,
                          delta.z * (beta.z * (lobe_value(sh.lobe, rho.z) * sh.G)));
            if (der != 0.0f) {
                ga[0] = delta.x * (beta.x * ((der * sh.G) * Le.x));
                ga[1] = delta.y * (beta.y * ((der * sh.G) * Le.y));
                ga[2] = delta.z * (beta.z * ((der * sh.G) * Le.z));
            }
        }
    }
    const bool cont = vo.cont;
    if (cont) {
        const float der = lobe_der(vo.scat);
        if (der != 0.0f) {
            const f3 rho = load3(sc.albedo, id);
            const float W[3] = {lobe_value(vo.scat, rho.x), lobe_value(vo.scat, rho.y), lobe_value(vo.scat, rho.z)};
            const float post[3] = {Ltot.x - ps.L.x, Ltot.y - ps.L.y, Ltot.z - ps.L.z};
            const float dl[3] = {delta.x, delta.y, delta.z};
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if (W[c] != 0.0f) ga[c] += dl[c] * (post[c] * (der / W[c]));
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) acc.add_tri(vo.hot, 0, c, g_alb + 3 * (size_t)id + c, ga[c]);
    if (!cont) return false;
    ar.pr.o = vo.o;
    ar.pr.d = vo.d;
    ++ar.pr.k;
    return true;
}

// The whole path: replay A, then replay B vertex by vertex.  With rec
// (records of path `path`), replay A keeps its intersections there and
// replay B reads them.
template <int LDS, bool ATTR = false, class Acc, bool COUNT = false>
PT_DEV void adjoint_path(const SceneView& sc, const CamView& cam, const PathParams& pp, uint32_t pix, uint32_t sample,
                         f3 delta, float* __restrict__ g_alb, float* __restrict__ g_emi, TravStack<LDS, COUNT>& st,
                         Acc& acc, const VertexRecs* rec = nullptr, uint32_t path = 0) {
    uint32_t ne = 0, ns = 0;
    AdjRun ar;
    if (rec) {
        PathRun pr;
        path_begin(cam, pp, pix, sample, pr);
        while (adjoint_a_vertex<LDS, ATTR>(sc, pp, pix, sample, path, pr, st, ne, ns, *rec)) {
        }
        adjoint_b_begin(cam, pp, pix, sample, delta, pr.ps.L, ar, path);
        while (adjoint_b_step<LDS, ATTR, Acc, COUNT, true>(sc, pp, ar, g_alb, g_emi, st, acc, ne, ns, *rec)) {
        }
        return;
    }
    const f3 Ltot = trace_path<LDS, COUNT, false, ATTR>(sc, cam, pp, pix, sample, st, ne, ns);
    adjoint_b_begin(cam, pp, pix, sample, delta, Ltot, ar);
    uint32_t be = 0, bs = 0;
    while (adjoint_b_step<LDS, ATTR>(sc, pp, ar, g_alb, g_emi, st, acc, be, bs)) {
    }
}

}  // namespace ptmi
