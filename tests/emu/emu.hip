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
    return v;
}

constexpr int kL = 16;

struct HostStack {
    uint32_t lref[kL];
    float lt[kL];
    std::vector<uint2> gbl;
    TravStack<kL> st;
    explicit HostStack(int gcap) : gbl(std::max(gcap, 1)) {
        st.lref = lref;
        st.lt = lt;
        st.lstride = 1;
        st.gbl = gbl.data();
        st.gstride = 1;
        st.gcap = gcap;
        st.sp = 0;
        st.overflow = false;
    }
};

}  // namespace

extern "C" {

// Megakernel body for the listed pixels: out[n*3].  rays[2] = extension
// and shadow ray counts.  Returns 0, or 1 if a traversal stack overflowed.
int32_t emu_render_mega(pt_ctx* c, const int32_t* pixels, int32_t n, int32_t spp, int32_t D, uint64_t seed,
                        uint32_t frame, uint32_t job, int32_t nee, int32_t rr_start, float* out, uint64_t* rays) {
    SceneView sc = host_view(c);
    PathParams pp{spp, D, nee ? 1 : 0, rr_start, seed, frame, job};
    HostStack hs(std::max(0, c->bvh.stack_entries - kL));
    uint64_t ne = 0, ns = 0;
    for (int32_t i = 0; i < n; ++i) {
        uint32_t pix = (uint32_t)pixels[i];
        uint32_t e = 0, s = 0;
        f3 sum = mk3(0.f, 0.f, 0.f);
        for (int k = 0; k < spp; ++k) {
            f3 L = trace_path<kL>(sc, c->cam, pp, pix, frame * (uint32_t)spp + (uint32_t)k, hs.st, e, s);
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

// Wavefront over the whole image: img[W*H*3]; shuffle_seed != 0 permutes
// every continuation and shadow queue.  compact = 0 keeps dead slots.
int32_t emu_render_wave(pt_ctx* c, int32_t spp, int32_t D, uint64_t seed, uint32_t frame, uint32_t job, int32_t nee,
                        int32_t rr_start, int32_t compact, uint64_t shuffle_seed, int32_t sort, float* img,
                        uint64_t* rays) {
    SceneView sc = host_view(c);
    PathParams pp{spp, D, nee ? 1 : 0, rr_start, seed, frame, job};
    const uint32_t npaths = (uint32_t)c->cam.W * c->cam.H * (uint32_t)spp;
    std::vector<float4> buf[11];
    for (auto& b : buf) b.assign(std::max<uint32_t>(npaths, 1), make_float4(0, 0, 0, 0));
    std::vector<uint32_t> counts((D + 2) + (D + 1) + 4, 0u);
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
    wb.sh_base = D + 2;
    wb.err_slot = (int)counts.size() - 1;
    std::mt19937_64 rng(shuffle_seed);
    HostStack hs(std::max(0, c->bvh.stack_entries - kL));
    counts[0] = npaths;
    for (uint32_t p = 0; p < npaths; ++p) raygen_item(c->cam, pp, wb, p);
    uint64_t ne = 0, ns = 0;
    for (int b = 0; b <= D; ++b) {
        const uint32_t count = counts[b];
        for (uint32_t i = 0; i < count; ++i) extend_item<kL>(sc, wb, b, i, hs.st);
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
        for (uint32_t i = 0; i < count; ++i) {
            VertexOut vo;
            ShadowReq sh;
            PathState ps;
            uint32_t path = shade_item(sc, pp, wb, b, i, vo, sh, ps, sort ? perm.data() : nullptr);
            if (path != kDeadPath) ++ne;
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
        for (uint32_t i = 0; i < nsh; ++i) shadow_item<kL>(sc, wb, i, hs.st);
        ns += nsh;
    }
    const uint32_t npix = (uint32_t)c->cam.W * c->cam.H;
    for (uint32_t pix = 0; pix < npix; ++pix) accumulate_item(pp, wb.L, img, nullptr, pix);
    rays[0] = ne;
    rays[1] = ns;
    return hs.st.overflow ? 1 : 0;
}

// Path-replay adjoint over the whole image (sequential binary32 adds):
// g_alb, g_emi (nt*3) are accumulated into.
int32_t emu_backward(pt_ctx* c, int32_t spp, int32_t D, uint64_t seed, uint32_t frame, uint32_t job, int32_t nee,
                     const float* d_img, float* g_alb, float* g_emi) {
    struct HostAcc {
        void add(float* p, float v) {
            if (v != 0.0f) *p += v;
        }
    } acc;
    SceneView sc = host_view(c);
    PathParams pp{spp, D, nee ? 1 : 0, -1, seed, frame, job};
    HostStack hs(std::max(0, c->bvh.stack_entries - kL));
    const uint32_t npaths = (uint32_t)c->cam.W * c->cam.H * (uint32_t)spp;
    const float fs = (float)spp;
    for (uint32_t p = 0; p < npaths; ++p) {
        const uint32_t pix = p / (uint32_t)spp, s = p - pix * (uint32_t)spp;
        f3 delta = mk3(d_img[3 * (size_t)pix] / fs, d_img[3 * (size_t)pix + 1] / fs, d_img[3 * (size_t)pix + 2] / fs);
        adjoint_path<kL>(sc, c->cam, pp, pix, frame * (uint32_t)spp + s, delta, g_alb, g_emi, hs.st, acc);
    }
    return hs.st.overflow ? 1 : 0;
}

}  // extern "C"
