// CPU emulator of the HIP path tracer, for tests only: the library's own
// device functions (traversal, shading, wavefront stage items) compiled for
// the host and driven sequentially.  The megakernel body runs per pixel; the
// wavefront runs stage by stage with a sequential queue counter in place of
// the wave ballots, optionally shuffling every queue to show that the result
// does not depend on queue order.
#include <algorithm>
#include <random>

#include "../../paper_2605_27323_amd/csrc/api.hip"
#include "../../paper_2605_27323_amd/csrc/wavefront.h"
#include "../../paper_2605_27323_amd/csrc/adjoint.h"
#include "../../paper_2605_27323_amd/csrc/batch.h"

namespace {

struct HostScene {
    SceneView v;
};

SceneView host_view(const pt_ctx* c) {
    SceneView v{};
    v.nodes = reinterpret_cast<const float4*>(c->bvh.nodes.data());
    v.tris = c->bvh.tris.data();
    v.lights = c->bvh.lights.data();
    v.mats = reinterpret_cast<const float4*>(c->mats.data());
    v.albedo = c->albedo.data();
    v.emission = c->emission.data();
    v.nl = (int32_t)c->bvh.lights.size();
    v.nt = c->nt;
    v.n_nodes = (int32_t)c->bvh.nodes.size();
    v.area_total = c->bvh.area_total;
    v.sky0 = c->sky[0];
    v.sky1 = c->sky[1];
    v.sky2 = c->sky[2];
    v.cx = c->bvh.center[0];
    v.cy = c->bvh.center[1];
    v.cz = c->bvh.center[2];
    v.hot_ids = c->bvh.hot_ids.data();
    v.n_hot = (int32_t)c->bvh.hot_ids.size();
    v.insts = c->bvh.insts.empty() ? nullptr : c->bvh.insts.data();
    v.n_inst = (int32_t)(c->bvh.insts.size() / kInstRecord);
    v.attrs = c->attr_leaf.empty() ? nullptr : c->attr_leaf.data();
    v.attr_flags = shading_flags(c);
    return v;
}

// the shading variant the library would launch
bool has_attrs(const pt_ctx* c) { return shading_flags(c) != 0; }

constexpr int kL = 16;

struct HostStack {
    uint2 l[kL + 1];
    std::vector<uint2> gbl;
    TravStack<kL> st;
    explicit HostStack(int gcap) : gbl(std::max(gcap, 1)) { st = make_trav_stack<kL>(l, 1, gbl.data(), 0u, 1, gcap); }
};

template <bool INST, bool ATTR>
int32_t render_mega(pt_ctx* c, const int32_t* pixels, int32_t n, int32_t spp, int32_t D, uint64_t seed,
                    uint32_t frame, uint32_t job, int32_t nee, int32_t rr_start, float* out, uint64_t* rays,
                    int32_t sampler) {
    SceneView sc = host_view(c);
    PathParams pp{spp, D, nee ? 1 : 0, rr_start, seed, frame, job, sampler};
    HostStack hs(std::max(0, c->bvh.stack_entries - kL));
    uint64_t ne = 0, ns = 0;
    for (int32_t i = 0; i < n; ++i) {
        uint32_t pix = (uint32_t)pixels[i];
        uint32_t e = 0, s = 0;
        f3 sum = mk3(0.f, 0.f, 0.f);
        for (int k = 0; k < spp; ++k) {
            f3 L = trace_path<kL, false, INST, ATTR>(sc, c->cam, pp, pix, frame * (uint32_t)spp + (uint32_t)k, hs.st, e,
                                                    s);
            sum = k == 0 ? L : add3(sum, L);
        }
        const float fs = (float)spp;
        out[3 * (size_t)i + 0] = sum.x / fs;
        out[3 * (size_t)i + 1] = sum.y / fs;
        out[3 * (size_t)i + 2] = sum.z / fs;
        ne += e;
        ns += s;
    }
    rays[0] = ne;
    rays[1] = ns;
    return hs.st.overflow ? 1 : 0;
}

}  // namespace

extern "C" {

// Megakernel body for the listed pixels: out[n*3].  rays[2] = extension
// and shadow ray counts.  Returns 0, or 1 if a traversal stack overflowed.
int32_t emu_render_mega(pt_ctx* c, const int32_t* pixels, int32_t n, int32_t spp, int32_t D, uint64_t seed,
                        uint32_t frame, uint32_t job, int32_t nee, int32_t rr_start, float* out, uint64_t* rays,
                        int32_t sampler) {
    // the kernel variant the library would launch for this scene
#define RM(I, A) render_mega<I, A>(c, pixels, n, spp, D, seed, frame, job, nee, rr_start, out, rays, sampler)
    const bool inst = !c->bvh.insts.empty();
    if (has_attrs(c)) return inst ? RM(true, true) : RM(false, true);
    return inst ? RM(true, false) : RM(false, false);
#undef RM
}

// Closest hit of the library's traversal for n rays o[3n], d[3n] in
// (0, inf): t, input triangle id (-1 on a miss), barycentrics.  Returns 1
// if a traversal stack overflowed.
int32_t emu_closest(pt_ctx* c, int32_t n, const float* o, const float* d, float* t, int32_t* id, float* b1,
                    float* b2) {
    SceneView sc = host_view(c);
    HostStack hs(std::max(0, c->bvh.stack_entries - kL));
    for (int32_t i = 0; i < n; ++i) {
        const f3 oo = mk3(o[3 * i], o[3 * i + 1], o[3 * i + 2]), dd = mk3(d[3 * i], d[3 * i + 1], d[3 * i + 2]);
        const Hit h = sc.n_inst > 0 ? closest_hit_t<kL, false, true>(sc, oo, dd, INFINITY, hs.st)
                                    : closest_hit<kL>(sc, make_ray(oo, dd), INFINITY, hs.st);
        t[i] = h.t;
        id[i] = h.tri == 0xFFFFFFFFu ? -1 : (int32_t)h.id;
        b1[i] = h.b1;
        b2[i] = h.b2;
    }
    return hs.st.overflow ? 1 : 0;
}

}  // extern "C"

namespace {

// The wavefront over the image; with rec, replay A of the adjoint with kept
// records (the path radiances then go to Lout).
template <bool INST, bool ATTR>
int32_t render_wave(pt_ctx* c, int32_t spp, int32_t D, uint64_t seed, uint32_t frame, uint32_t job, int32_t nee,
                    int32_t rr_start, int32_t compact, uint64_t shuffle_seed, int32_t sort, uint32_t tail,
                    float* img, uint64_t* rays, int32_t sampler, const VertexRecs* rec = nullptr,
                    float4* Lout = nullptr) {
    SceneView sc = host_view(c);
    PathParams pp{spp, D, nee ? 1 : 0, rr_start, seed, frame, job, sampler};
    const uint32_t npaths = (uint32_t)c->cam.W * c->cam.H * (uint32_t)spp;
    std::vector<float4> buf[11];
    for (auto& b : buf) b.assign(std::max<uint32_t>(npaths, 1), make_float4(0, 0, 0, 0));
    std::vector<uint32_t> counts(2 * D + 6, 0u);
    WaveBufs wb{};
    for (int q = 0; q < 2; ++q) {
        wb.ray_o[q] = buf[0 + q].data();
        wb.ray_d[q] = buf[2 + q].data();
        wb.pst[q] = buf[4 + q].data();
    }
    wb.hit = buf[6].data();
    wb.sh_o = buf[7].data();
    wb.sh_d = buf[8].data();
    wb.sh_c = buf[9].data();
    wb.L = buf[10].data();
    wb.counts = counts.data();
    if (rec) {
        wb.rec_hit = rec->hit;
        wb.rec_vis = rec->vis;
        wb.rec_n = rec->npaths;
    }
    wb.sh_base = D + 2;
    wb.tail_slot = 2 * D + 3;
    wb.err_slot = (int)counts.size() - 1;
    std::mt19937_64 rng(shuffle_seed);
    HostStack hs(std::max(0, c->bvh.stack_entries - kL));
    counts[0] = npaths;
    for (uint32_t p = 0; p < npaths; ++p) raygen_item(c->cam, pp, wb, p);
    uint64_t ne = 0, ns = 0;
    for (int b = 0; b <= D; ++b) {
        const uint32_t count = counts[b];
        for (uint32_t i = 0; i < count; ++i) extend_item<kL, false, INST>(sc, wb, b, i, hs.st);
        const int nxt = (b & 1) ^ 1;
        // material sort: counting sort of the slots by key (ties in slot order)
        std::vector<uint32_t> perm;
        if (sort) {
            std::vector<uint32_t> key(count), off(kSortBins + 1, 0u);
            for (uint32_t i = 0; i < count; ++i) {
                key[i] = material_key(sc, wb.hit[i]);
                off[key[i] + 1]++;
            }
            for (int t = 0; t < kSortBins; ++t) off[t + 1] += off[t];
            perm.resize(count);
            for (uint32_t i = 0; i < count; ++i) perm[off[key[i]]++] = i;
            for (uint32_t i = 1; i < count; ++i)  // keys are non-decreasing along perm
                if (material_key(sc, wb.hit[perm[i]]) < material_key(sc, wb.hit[perm[i - 1]])) return 2;
        }
        const bool finish = compact && count < tail;
        for (uint32_t i = 0; i < count; ++i) {
            VertexOut vo;
            ShadowReq sh;
            PathState ps;
            uint32_t path = shade_item<INST, ATTR>(sc, pp, wb, b, i, vo, sh, ps, sort ? perm.data() : nullptr,
                                             no_light_cache(), finish);
            if (path != kDeadPath) ++ne;
            if (finish) {
                uint32_t te = 0, ts = 0;
                finish_path<kL, false, INST, ATTR>(sc, pp, wb, path, b + 1, vo, sh, ps, hs.st, te, ts);
                ne += te;
                ns += ts;
                continue;
            }
            if (compact) {
                if (vo.cont) write_continuation(wb, nxt, counts[b + 1]++, vo, ps, path);
            } else {
                if (vo.cont) write_continuation(wb, nxt, i, vo, ps, path);
                else write_dead(wb, nxt, i);
            }
            if (sh.valid) write_shadow(wb, counts[wb.sh_base + b]++, sh, path);
        }
        if (!compact) counts[b + 1] = count;
        const uint32_t nsh = counts[wb.sh_base + b];
        if (shuffle_seed) {
            std::vector<uint32_t> perm(counts[b + 1]);
            for (uint32_t i = 0; i < perm.size(); ++i) perm[i] = i;
            std::shuffle(perm.begin(), perm.end(), rng);
            for (int f = 0; f < 3; ++f) {
                std::vector<float4>& v = buf[2 * f + nxt];
                std::vector<float4> tmp(v.begin(), v.begin() + perm.size());
                for (uint32_t i = 0; i < perm.size(); ++i) v[i] = tmp[perm[i]];
            }
            std::vector<uint32_t> ps(nsh);
            for (uint32_t i = 0; i < nsh; ++i) ps[i] = i;
            std::shuffle(ps.begin(), ps.end(), rng);
            for (int f = 7; f <= 9; ++f) {
                std::vector<float4> tmp(buf[f].begin(), buf[f].begin() + nsh);
                for (uint32_t i = 0; i < nsh; ++i) buf[f][i] = tmp[ps[i]];
            }
        }
        for (uint32_t i = 0; i < nsh; ++i) shadow_item<kL, false, INST>(sc, wb, b, i, hs.st);
        ns += nsh;
    }
    const uint32_t npix = (uint32_t)c->cam.W * c->cam.H;
    if (Lout) std::copy(buf[10].begin(), buf[10].begin() + npaths, Lout);
    if (img)
        for (uint32_t pix = 0; pix < npix; ++pix) accumulate_item(pp, wb.L, img, nullptr, pix);
    rays[0] = ne;
    rays[1] = ns;
    return hs.st.overflow ? 1 : 0;
}

}  // namespace

extern "C" {

// Wavefront over the whole image: img[W*H*3]; shuffle_seed != 0 permutes
// every continuation and shadow queue.  compact = 0 keeps dead slots.
int32_t emu_render_wave(pt_ctx* c, int32_t spp, int32_t D, uint64_t seed, uint32_t frame, uint32_t job, int32_t nee,
                        int32_t rr_start, int32_t compact, uint64_t shuffle_seed, int32_t sort, uint32_t tail,
                        float* img, uint64_t* rays, int32_t sampler) {
#define RW(I, A) \
    render_wave<I, A>(c, spp, D, seed, frame, job, nee, rr_start, compact, shuffle_seed, sort, tail, img, rays, sampler)
    const bool inst = !c->bvh.insts.empty();
    if (has_attrs(c)) return inst ? RW(true, true) : RW(false, true);
    return inst ? RW(true, false) : RW(false, false);
#undef RW
}

// Path-replay adjoint over the whole image (sequential binary32 adds):
// g_alb, g_emi (nt*3) are accumulated into.  keep_hits: replay A keeps
// every vertex's intersection and light-sample visibility and replay B
// reads them (the records of all paths, laid out as the GPU's); 1: replay
// A path by path (megakernel order), 2: replay A as the wavefront over all
// paths first (queues shuffled), 3: as 2 with every path finished by the
// hybrid tail from its first vertex on.
int32_t emu_backward(pt_ctx* c, int32_t spp, int32_t D, uint64_t seed, uint32_t frame, uint32_t job, int32_t nee,
                     const float* d_img, float* g_alb, float* g_emi, int32_t sampler, int32_t keep_hits) {
    struct HostAcc {
        void add(float* p, float v) {
            if (v != 0.0f) *p += v;
        }
        void add_tri(uint32_t, int, int, float* p, float v) { add(p, v); }
        void add_light(uint32_t, int, float* p, float v) { add(p, v); }
    } acc;
    SceneView sc = host_view(c);
    PathParams pp{spp, D, nee ? 1 : 0, -1, seed, frame, job, sampler};
    HostStack hs(std::max(0, c->bvh.stack_entries - kL));
    const uint32_t npaths = (uint32_t)c->cam.W * c->cam.H * (uint32_t)spp;
    const float fs = (float)spp;
    const size_t nrec = keep_hits ? (size_t)npaths * ((size_t)std::max(D, 0) + 1) : 0;
    // records filled with a pattern, so that a read of a slot replay A did
    // not write would show
    std::vector<uint2> hits(nrec, make_uint2(0x7FC00001u, 0xFFFFFFFEu));
    std::vector<uint8_t> vis(nrec, 0x5Au);
    const VertexRecs rec{hits.data(), vis.data(), npaths};
    if (keep_hits >= 2) {
        std::vector<float4> L(std::max<uint32_t>(npaths, 1));
        uint64_t rays[2];
        const uint32_t tail = keep_hits == 3 ? npaths + 1 : 0u;
        const int32_t rc = has_attrs(c) ? render_wave<false, true>(c, spp, D, seed, frame, job, nee, -1, 1, 77, 0, tail,
                                                                   nullptr, rays, sampler, &rec, L.data())
                                        : render_wave<false, false>(c, spp, D, seed, frame, job, nee, -1, 1, 77, 0,
                                                                    tail, nullptr, rays, sampler, &rec, L.data());
        if (rc) return rc;
        for (uint32_t p = 0; p < npaths; ++p) {
            const uint32_t pix = p / (uint32_t)spp, s = p - pix * (uint32_t)spp;
            f3 delta =
                mk3(d_img[3 * (size_t)pix] / fs, d_img[3 * (size_t)pix + 1] / fs, d_img[3 * (size_t)pix + 2] / fs);
            AdjRun ar;
            adjoint_b_begin(c->cam, pp, pix, frame * (uint32_t)spp + s, delta, xyz(L[p]), ar, p);
            uint32_t ne = 0, ns = 0;
            if (has_attrs(c)) {
                while (adjoint_b_step<kL, true, HostAcc, false, true>(sc, pp, ar, g_alb, g_emi, hs.st, acc, ne, ns, rec)) {
                }
            } else {
                while (adjoint_b_step<kL, false, HostAcc, false, true>(sc, pp, ar, g_alb, g_emi, hs.st, acc, ne, ns, rec)) {
                }
            }
        }
        return hs.st.overflow ? 1 : 0;
    }
    for (uint32_t p = 0; p < npaths; ++p) {
        const uint32_t pix = p / (uint32_t)spp, s = p - pix * (uint32_t)spp;
        f3 delta = mk3(d_img[3 * (size_t)pix] / fs, d_img[3 * (size_t)pix + 1] / fs, d_img[3 * (size_t)pix + 2] / fs);
        const VertexRecs* r = keep_hits ? &rec : nullptr;
        if (has_attrs(c))
            adjoint_path<kL, true>(sc, c->cam, pp, pix, frame * (uint32_t)spp + s, delta, g_alb, g_emi, hs.st, acc, r, p);
        else
            adjoint_path<kL, false>(sc, c->cam, pp, pix, frame * (uint32_t)spp + s, delta, g_alb, g_emi, hs.st, acc, r, p);
    }
    return hs.st.overflow ? 1 : 0;
}

// Batched pool over the jobs (host memory copies of the scenes), images
// written job after job into img (concatenated W*H*3 blocks).  Returns the
// number of iterations, or -1 on a bookkeeping error.
int64_t emu_render_batch(pt_ctx** ctxs, const pt_render_args* args, int32_t n, uint32_t capacity, uint64_t shuffle_seed,
                         float* img) {
    std::vector<JobDesc> jobs(n);
    uint64_t total = 0, total_pix = 0;
    bool any_attr = false;
    for (int j = 0; j < n; ++j) any_attr = any_attr || has_attrs(ctxs[j]);
    int gcap = 0;
    for (int j = 0; j < n; ++j) {
        JobDesc& d = jobs[j];
        d.sc = host_view(ctxs[j]);
        d.cam = ctxs[j]->cam;
        d.pp = PathParams{args[j].spp, args[j].max_depth, args[j].nee ? 1 : 0, args[j].rr_start, args[j].seed,
                          args[j].frame, args[j].job, args[j].sampler};
        d.npix = (uint32_t)d.cam.W * d.cam.H;
        d.npaths = d.npix * (uint32_t)args[j].spp;
        d.img = img + 3 * total_pix;
        d.base = (uint32_t)total;
        d.pix_base = (uint32_t)total_pix;
        total += d.npaths;
        total_pix += d.npix;
        gcap = std::max(gcap, ctxs[j]->bvh.stack_entries - kL);
    }
    std::vector<float4> pool(10 * (size_t)capacity), L(std::max<uint64_t>(total, 1));
    std::vector<uint32_t> remaining(n);
    std::vector<uint64_t> done_ts(n);
    BatchCtl ctl{};
    BatchBufs bb{};
    bb.jobs = jobs.data();
    bb.njobs = n;
    bb.capacity = capacity;
    bb.ctl = &ctl;
    bb.remaining = remaining.data();
    bb.done_ts = done_ts.data();
    const size_t C = capacity;
    bb.ray_o[0] = &pool[0]; bb.ray_o[1] = &pool[C];
    bb.ray_d[0] = &pool[2 * C]; bb.ray_d[1] = &pool[3 * C];
    bb.pst[0] = &pool[4 * C]; bb.pst[1] = &pool[5 * C];
    bb.hit = &pool[6 * C];
    bb.sh_o = &pool[7 * C]; bb.sh_d = &pool[8 * C]; bb.sh_c = &pool[9 * C];
    bb.L = L.data();
    ctl.total = (uint32_t)total;
    for (int j = 0; j < n; ++j) remaining[j] = jobs[j].npaths;
    HostStack hs(std::max(0, gcap));
    std::mt19937_64 rng(shuffle_seed);
    int64_t it = 0;
    for (;; ++it) {
        const int q = (int)(it & 1);
        batch_schedule(bb, q);
        if (ctl.done) break;
        if (it > 100000000) return -1;
        for (uint32_t i = 0; i < ctl.regen_n; ++i) batch_regen_item(bb, q, i);
        for (uint32_t i = 0; i < ctl.count; ++i) batch_extend_item<kL>(bb, q, i, hs.st);
        for (uint32_t i = 0; i < ctl.count; ++i) {
            VertexOut vo;
            ShadowReq sh;
            PathState ps;
            uint32_t g = 0, meta = 0;
            bool fin = any_attr ? batch_shade_item<true>(bb, q, i, vo, sh, ps, g, meta)
                                : batch_shade_item<false>(bb, q, i, vo, sh, ps, g, meta);
            if (fin && remaining[meta >> 24]-- == 0) return -1;
            if (vo.cont) {
                if (ctl.live[q ^ 1] >= capacity) return -1;
                batch_write_continuation(bb, q ^ 1, ctl.live[q ^ 1]++, vo, ps, g, meta);
            }
            if (sh.valid) batch_write_shadow(bb, ctl.shadow++, sh, g, meta >> 24, !vo.cont);
        }
        if (shuffle_seed) {  // queue order must not matter
            std::vector<uint32_t> perm(ctl.shadow);
            for (uint32_t i = 0; i < perm.size(); ++i) perm[i] = i;
            std::shuffle(perm.begin(), perm.end(), rng);
            for (float4* f : {bb.sh_o, bb.sh_d, bb.sh_c}) {
                std::vector<float4> tmp(f, f + perm.size());
                for (uint32_t i = 0; i < perm.size(); ++i) f[i] = tmp[perm[i]];
            }
        }
        for (uint32_t i = 0; i < ctl.shadow; ++i) {
            uint32_t job = 0;
            if (batch_shadow_item<kL>(bb, i, hs.st, job) && remaining[job]-- == 0) return -1;
        }
    }
    for (int j = 0; j < n; ++j)
        if (remaining[j] != 0) return -1;
    for (uint32_t gp = 0; gp < total_pix; ++gp) batch_accumulate_item(bb, gp);
    return it;
}

}  // extern "C"
