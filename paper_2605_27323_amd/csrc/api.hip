// C-ABI entry points of libptmi (declared in include/ptmi.h).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "batch.h"
#include "bvh_build.h"
#include "kernels.h"
#include "noalloc.h"

using namespace ptmi;

namespace {

thread_local std::string g_err;

pt_status fail(pt_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

pt_status hip_fail(hipError_t e, const char* what) {
    return fail(PT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define PT_HIP(call, what)                            \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// frames in flight in pt_render_frames (internal streams and workspace
// slots): one stream per frame, each on a hardware queue of its own beside
// the caller's and one to spare; HIP gives a process GPU_MAX_HW_QUEUES of
// them (4 unless the environment says otherwise), so the count follows that
// setting, from 3 up to kMaxInFlight.  Sharing queues cost more than the
// extra frame gained (measured with eight queues: 5 frames 1.61, 6 frames
// 1.59, 7 frames 1.80 ms per frame; 8 frames with ten queues 1.57).
constexpr int kMaxInFlight = 8;
int frames_in_flight_for_queues() {
    const char* e = std::getenv("GPU_MAX_HW_QUEUES");
    const int q = e && *e ? std::atoi(e) : 4;
    return std::max(3, std::min(kMaxInFlight, q - 2));
}
constexpr int kDefaultBlock = 256;
constexpr int kDefaultGridMult = 8;
constexpr int kStackLds = 8;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }
constexpr int kMaxPools = 4;  // concurrent pools of a batched launch
constexpr uint32_t kTailWavesPerCu = 16;  // the hybrid tail kernel runs 4 waves per SIMD

struct StageTimer {
    int stage;
    hipEvent_t a, b;
};

}  // namespace

struct pt_ctx {
    int device = -1;
    int num_cu = 256;
    size_t lds_per_block = 160 * 1024;  // LDS a workgroup may allocate on this device
    // scene (host copy)
    bool loaded = false, built = false, bound = false, cam_set = false;
    int32_t nt = 0, nm = 0;
    std::vector<float> tri_v, albedo, emission, mats;
    std::vector<int32_t> tri_mat;
    float sky[3] = {0, 0, 0};
    BuildResult bvh;
    InstanceSet inst;  // two-level scene (no instances: flat)
    // vertex attributes per triangle corner (input order; empty = none):
    // normals nt * 9, texture coordinates nt * 6; attr_leaf: the device
    // records in leaf order (kAttrRecord float4 per triangle)
    int32_t nv = 0;
    std::vector<int32_t> tri_idx;
    std::vector<float> attr_n, attr_uv;
    std::vector<float4> attr_leaf;
    SceneView view{};
    CamView cam{};
    // profiling
    std::vector<StageTimer> timers;
    std::vector<hipEvent_t> event_pool;
    size_t event_next = 0;
    // last frame: device counters and what is needed to turn them into
    // per-stage work items and bytes
    // frames in flight (pt_render_frames): internal streams and their
    // events, created on first use
    bool aux_ready = false;
    int in_flight = 3;  // frames in flight (set at creation)
    hipStream_t aux[kMaxInFlight] = {};
    hipEvent_t ev_entry = nullptr, ev_stage[kMaxInFlight] = {}, ev_acc[kMaxInFlight] = {};
    // a single wavefront frame: the side stream that runs each bounce's
    // shadow stage beside the next extend stage, and its fork / join events
    // (two per bounce), created on first use
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> side_ev;
    uint32_t* last_counts = nullptr;
    unsigned long long* last_trav = nullptr;
    int last_ncounts = 0, last_D = 0, last_kind = 0;  // kind: 0 megakernel, 1 wavefront, 2 adjoint
    int last_spp = 1, last_nee = 1, last_compact = 1, last_sort = 0;
    uint32_t last_tail = 0, last_sort_threshold = 0;
    int last_tail_bounce = 0;
    int64_t last_promotes = 0;  // promote launches of the last frame (PT_FLAG_TWO_SLOT)
    bool last_replay_wave = false;  // the last backward ran replay A as the wavefront
    uint32_t* last_ovf_a = nullptr;  // then: the wavefront stages' overflow flag
    bool last_keep_hits = false;     // the last backward kept replay A's intersections
    uint64_t last_npix = 0;
    bool last_acc = false;
    bool last_valid = false;
};

namespace {

// LDS stack entries per lane: requested (8, 16, 24, 32) or the default,
// never more than the BVH can need; the block's stacks plus the largest
// static LDS of a traversal kernel (the light table) must fit a workgroup
int stack_lds_for(int requested, int need, int block, size_t lds_per_block, int& out) {
    int lds = requested > 0 ? requested : kStackLds;
    if (lds != 8 && lds != 16 && lds != 24 && lds != 32) return fail(PT_EINVAL, "stack_lds must be 8, 16, 24 or 32");
    while (lds > 8 && lds - 8 >= need) lds -= 8;
    if (trav_stack_lds_bytes(lds, block) + 3 * sizeof(uint32_t) * kLdsLights > lds_per_block)
        return fail(PT_EINVAL, "stack_lds x block exceeds the LDS of a workgroup");
    out = lds;
    return PT_OK;
}

struct Launch {
    int block, grid;
    int lds;
    int gcap;
    uint32_t nlanes;
};

pt_status launch_config(const pt_ctx* c, const pt_render_args* a, Launch& L) {
    L.block = a->block > 0 ? a->block : kDefaultBlock;
    int mult = a->grid_mult > 0 ? a->grid_mult : kDefaultGridMult;
    if (L.block < 64 || L.block > 256 || (L.block % 64) != 0) return fail(PT_EINVAL, "block must be a multiple of 64 in [64, 256]");
    if (mult < 1 || mult > 64) return fail(PT_EINVAL, "grid_mult must be in [1, 64]");
    L.grid = c->num_cu * mult;
    pt_status st = stack_lds_for(a->stack_lds, c->bvh.stack_entries, L.block, c->lds_per_block, L.lds);
    if (st) return st;
    L.gcap = std::max(0, c->bvh.stack_entries - L.lds);
    L.nlanes = (uint32_t)L.grid * (uint32_t)L.block;
    return PT_OK;
}

struct WsLayout {
    size_t counts, trav, ovf, ovf2, adj, rec_hit, rec_vis, wave[11], sort_key, perm, hist, total;
    int ncounts;
};
constexpr int kTravWords = 16;  // 8 u64 traversal work counters

// workspace: counters | traversal overflow stack | adjoint path cursors and
// radiance (backward only) | wavefront state (wavefront only)
WsLayout layout(const pt_ctx* c, const pt_render_args* a, const Launch& L, bool backward = false) {
    WsLayout w{};
    const size_t npaths = (size_t)c->cam.W * c->cam.H * a->spp;
    // [0, D+1] live paths per bounce, [D+2, 2D+2] shadow rays per bounce,
    // [2D+3, 2D+4] rays traced by the hybrid tail, [2D+6, 2D+7] the
    // two-slot count buffer (PT_FLAG_TWO_SLOT), the last word the overflow flag
    // (the megakernel's eight band cursors, u64, take words 8 .. 23)
    w.ncounts = std::max(2 * a->max_depth + 9, 24);
    size_t off = 0;
    w.counts = off;
    off = align_up(off + sizeof(uint32_t) * w.ncounts);
    w.trav = off;
    off = align_up(off + sizeof(uint32_t) * kTravWords);
    w.ovf = off;
    off = align_up(off + sizeof(uint2) * (size_t)L.gcap * L.nlanes);
    // the wavefront's shadow stage runs beside the next extend stage (on the
    // context's side stream) and spills its stacks to an area of its own
    const bool wave_mode = a->mode == PT_MODE_WAVE;
    w.ovf2 = off;
    if (wave_mode) off = align_up(off + sizeof(uint2) * (size_t)L.gcap * L.nlanes);
    // the adjoint's two path cursors and replay B's counters (one aligned
    // block), then the per-path radiance when replay A runs as the
    // megakernel-style kernel (as the wavefront it is the wavefront's
    // per-path radiance buffer)
    const bool wave = a->mode == PT_MODE_WAVE;
    w.adj = off;
    if (backward) off = align_up(off + kAlign + (wave ? 0 : sizeof(float4) * npaths));
    // PT_FLAG_KEEP_HITS: replay A's records, max_depth + 1 vertices per path
    const bool keep = backward && (a->flags & PT_FLAG_KEEP_HITS) != 0;
    const size_t nrec = npaths * ((size_t)std::max(a->max_depth, 0) + 1);
    w.rec_hit = off;
    if (keep) off = align_up(off + sizeof(uint2) * nrec);
    w.rec_vis = off;
    if (keep) off = align_up(off + nrec);
    for (int i = 0; i < 11; ++i) {
        w.wave[i] = off;
        if (wave) off = align_up(off + sizeof(float4) * npaths);
    }
    w.sort_key = off;
    if (wave) off = align_up(off + sizeof(uint32_t) * npaths);
    w.perm = off;
    if (wave) off = align_up(off + sizeof(uint32_t) * npaths);
    w.hist = off;
    if (wave) off = align_up(off + sizeof(uint32_t) * (2 * kSortBins + 1));
    w.total = off;
    return w;
}

pt_status check_args(const pt_ctx* c, const pt_render_args* a) {
    if (!c) return fail(PT_EINVAL, "null context");
    if (!a) return fail(PT_EINVAL, "null args");
    if (c->device < 0) return fail(PT_ESTATE, "host-only context cannot render");
    if (!c->bound) return fail(PT_ESTATE, "scene not bound (pt_bind_scene)");
    if (!c->cam_set) return fail(PT_ESTATE, "camera not set (pt_set_camera)");
    if (a->flags & ~(PT_FLAG_PROFILE | PT_FLAG_NO_COMPACT | PT_FLAG_SORT_MATERIAL | PT_FLAG_COUNT_WORK | PT_FLAG_SORT_RAYS |
                     PT_FLAG_XCD_LOCAL | PT_FLAG_TWO_SLOT | PT_FLAG_KEEP_HITS | PT_FLAG_SERIAL_STAGES))
        return fail(PT_EINVAL, "unknown flag");
    if (a->spp < 1 || a->spp > 65536) return fail(PT_EINVAL, "spp must be in [1, 65536]");
    if (a->max_depth < 0 || a->max_depth > 1000) return fail(PT_EINVAL, "max_depth must be in [0, 1000]");
    if (a->tail_bounce < 0 || a->tail_bounce > a->max_depth)
        return fail(PT_EINVAL, "tail_bounce must be in [0, max_depth]");
    if (a->tail_spread != 0 && a->tail_spread != 1) return fail(PT_EINVAL, "tail_spread must be 0 or 1");
    if (a->mega_waves != 0 && a->mega_waves != 4 && a->mega_waves != 5)
        return fail(PT_EINVAL, "mega_waves must be 0, 4 or 5");
    if (a->sampler != PT_SAMPLER_PHILOX && a->sampler != PT_SAMPLER_HALTON)
        return fail(PT_EINVAL, "sampler must be PT_SAMPLER_PHILOX or PT_SAMPLER_HALTON");
    if (a->mode != PT_MODE_MEGA && a->mode != PT_MODE_WAVE) return fail(PT_EINVAL, "unknown mode");
    const uint64_t npaths = (uint64_t)c->cam.W * c->cam.H * a->spp;
    if (npaths >= 0xFFFFFFFFull) return fail(PT_EINVAL, "width * height * spp must be < 2^32 - 1");
    return PT_OK;
}

hipEvent_t next_event(pt_ctx* c) {
    if (c->event_next == c->event_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->event_pool.push_back(e);
    }
    return c->event_pool[c->event_next++];
}

// run `fn` (a launch) bracketed by events when profiling
template <typename F>
hipError_t timed(pt_ctx* c, bool prof, int stage, hipStream_t s, F fn) {
    if (!prof) return fn();
    StageTimer t{stage, next_event(c), next_event(c)};
    if (!t.a || !t.b) return hipErrorOutOfMemory;
    (void)hipEventRecord(t.a, s);
    hipError_t e = fn();
    (void)hipEventRecord(t.b, s);
    c->timers.push_back(t);
    return e;
}

void remember_frame(pt_ctx* c, const pt_render_args* a, uint32_t* counts, int ncounts, int kind, bool acc,
                    int64_t promotes = 0) {
    c->last_counts = counts;
    c->last_promotes = promotes;
    c->last_ncounts = ncounts;
    c->last_D = a->max_depth;
    c->last_kind = kind;
    c->last_spp = a->spp;
    c->last_nee = a->nee ? 1 : 0;
    c->last_compact = (a->flags & PT_FLAG_NO_COMPACT) ? 0 : 1;
    c->last_sort = ((a->flags & PT_FLAG_SORT_MATERIAL) ? 1 : 0) + ((a->flags & PT_FLAG_SORT_RAYS) ? 1 : 0);
    c->last_tail = a->tail_threshold;
    c->last_tail_bounce = a->tail_bounce;
    c->last_sort_threshold = a->sort_threshold;
    c->last_npix = (uint64_t)c->cam.W * (uint64_t)c->cam.H;
    c->last_acc = acc;
    c->last_valid = true;
}

// bytes of one frame's workspace slot in pt_render_frames: the frame
// layout plus the frame's image (the megakernel writes it there)
size_t frame_slot_bytes(const pt_ctx* c, const WsLayout& w) {
    return align_up(w.total + sizeof(float) * 3 * (size_t)c->cam.W * (size_t)c->cam.H);
}

// The side stream of a context and at least nev fork / join events.
pt_status side_stream(pt_ctx* c, int nev, hipStream_t& out) {
    if (!c->side) PT_HIP(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking), "create stream");
    while ((int)c->side_ev.size() < nev) {
        hipEvent_t e = nullptr;
        PT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "create event");
        c->side_ev.push_back(e);
    }
    out = c->side;
    return PT_OK;
}

// Enqueue one frame on stream s, except the wavefront's accumulate (its
// radiance buffer is returned in *Lbuf): counters, then the megakernel
// (writing img / acc) or raygen and the bounce stages.  With s2 (the
// wavefront only), each bounce's shadow stage runs on s2, beside the next
// bounce's extend stage on s: they read and write disjoint buffers (the
// shadow records and the path radiance, the next rays and their hits), and
// the next shade stage, which adds to the radiance and overwrites the
// shadow records,
// waits for it.  The image is the same bit for bit.
pt_status enqueue_stages(pt_ctx* c, const pt_render_args* a, const Launch& L, const WsLayout& w, char* base,
                         hipStream_t s, float* img, float* acc, bool prof, const float4** Lbuf,
                         const VertexRecs* rec = nullptr, hipStream_t s2 = nullptr) {
    uint32_t* counts = reinterpret_cast<uint32_t*>(base + w.counts);
    unsigned long long* trav = reinterpret_cast<unsigned long long*>(base + w.trav);
    uint2* ovf = reinterpret_cast<uint2*>(base + w.ovf);
    PathParams pp{a->spp, a->max_depth, a->nee ? 1 : 0, a->rr_start, a->seed, a->frame, a->job, a->sampler};
    dim3 grid(L.grid), block(L.block);
    const bool count = (a->flags & PT_FLAG_COUNT_WORK) != 0;
    const int xcd = (a->flags & PT_FLAG_XCD_LOCAL) ? 1 : 0;
    PT_HIP(launch_init_counts(s, reinterpret_cast<uint32_t*>(trav), kTravWords, 0u), "init work counters");
    const uint32_t npaths = (uint32_t)c->cam.W * c->cam.H * a->spp;
    if (a->mode == PT_MODE_MEGA) {
        PT_HIP(launch_init_counts(s, counts, w.ncounts, 0u), "init counters");
        // counters: [0] extension rays, [1] shadow rays, [2] overflow flag, [4..5] the
        // megakernel's 64-bit pixel cursor
        PT_HIP(timed(c, prof, 5, s, [&] { return launch_mega(L.lds, count, a->mega_waves == 5 ? 5 : 4, grid, block, s, c->view, c->cam, pp, img, acc, ovf, L.gcap, counts, trav, xcd); }), "megakernel");
        remember_frame(c, a, counts, w.ncounts, 0, acc != nullptr);
    } else {
        WaveBufs wb{};
        for (int q = 0; q < 2; ++q) {
            wb.ray_o[q] = reinterpret_cast<float4*>(base + w.wave[0 + q]);
            wb.ray_d[q] = reinterpret_cast<float4*>(base + w.wave[2 + q]);
            wb.pst[q] = reinterpret_cast<float4*>(base + w.wave[4 + q]);
        }
        wb.hit = reinterpret_cast<float4*>(base + w.wave[6]);
        wb.sh_o = reinterpret_cast<float4*>(base + w.wave[7]);
        wb.sh_d = reinterpret_cast<float4*>(base + w.wave[8]);
        wb.sh_c = reinterpret_cast<float4*>(base + w.wave[9]);
        wb.L = reinterpret_cast<float4*>(base + w.wave[10]);
        wb.counts = counts;
        wb.trav = trav;
        wb.sh_base = a->max_depth + 2;
        wb.tail_slot = 2 * a->max_depth + 3;
        wb.err_slot = w.ncounts - 1;
        wb.two_slot = (a->flags & PT_FLAG_TWO_SLOT) ? 1 : 0;
        wb.slot = 2 * a->max_depth + 6;
        wb.sort_key = reinterpret_cast<uint32_t*>(base + w.sort_key);
        wb.perm = reinterpret_cast<uint32_t*>(base + w.perm);
        wb.hist = reinterpret_cast<uint32_t*>(base + w.hist);
        if (rec) {
            wb.rec_hit = rec->hit;
            wb.rec_vis = rec->vis;
            wb.rec_n = rec->npaths;
        }
        const int compact = (a->flags & PT_FLAG_NO_COMPACT) ? 0 : 1;
        const int sort = (a->flags & PT_FLAG_SORT_MATERIAL) ? 1 : 0;
        const int rsort = (a->flags & PT_FLAG_SORT_RAYS) ? 1 : 0;
        if ((sort || rsort) && !compact) return fail(PT_EINVAL, "sorting needs compaction");
        PT_HIP(launch_init_counts(s, counts, w.ncounts, npaths), "init counters");
        if (sort || rsort) PT_HIP(launch_init_counts(s, wb.hist, 2 * kSortBins + 1, 0u), "init sort histogram");
        PT_HIP(timed(c, prof, 0, s, [&] { return launch_raygen(grid, block, s, c->cam, pp, wb); }), "raygen");
        uint2* ovf2 = reinterpret_cast<uint2*>(base + w.ovf2);
        const bool fork = s2 != nullptr && a->nee;
        int pend = -1;  // bounce whose shadow stage runs on s2, not yet joined
        int64_t promotes = 0;
        if (wb.two_slot) {
            PT_HIP(timed(c, prof, 10, s, [&] { return launch_promote(s, wb, -1); }), "promote");
            ++promotes;
        }
        for (int b = 0; b <= a->max_depth; ++b) {
            if (rsort)
                PT_HIP(timed(c, prof, 6, s, [&] { return launch_sort(grid, block, s, c->view, wb, b, a->sort_threshold, 1); }), "ray sort");
            PT_HIP(timed(c, prof, 1, s, [&] { return launch_extend(L.lds, count, grid, block, s, c->view, wb, b, ovf, L.gcap, rsort, xcd); }), "extend");
            if (sort)
                PT_HIP(timed(c, prof, 6, s, [&] { return launch_sort(grid, block, s, c->view, wb, b, a->sort_threshold, 0); }), "sort");
            // at bounce tail_bounce the hybrid tail takes whatever is left
            // (threshold above any queue size); later bounces have nothing
            const bool last = compact && a->tail_bounce > 0 && b == a->tail_bounce;
            const uint32_t tail = last ? 0xFFFFFFFFu : a->tail_threshold;
            if (pend >= 0) {
                PT_HIP(hipStreamWaitEvent(s, c->side_ev[2 * pend + 1], 0), "join shadow stage");
                pend = -1;
            }
            PT_HIP(timed(c, prof, 2, s, [&] { return launch_shade(grid, block, s, c->view, pp, wb, b, compact, sort, tail); }), "shade");
            if (compact && tail)
                PT_HIP(timed(c, prof, 8, s, [&] {
                           return launch_tail(L.lds, count, grid, block, s, c->view, pp, wb, b, sort, tail, ovf, L.gcap,
                                              a->tail_spread ? (uint32_t)c->num_cu * kTailWavesPerCu : 0u);
                       }),
                       "hybrid tail");
            if (last) break;
            if (wb.two_slot) {
                PT_HIP(timed(c, prof, 10, s, [&] { return launch_promote(s, wb, b); }), "promote");
                ++promotes;
            }
            if (b < a->max_depth && a->nee) {
                if (fork) {
                    PT_HIP(hipEventRecord(c->side_ev[2 * b], s), "fork shadow stage");
                    PT_HIP(hipStreamWaitEvent(s2, c->side_ev[2 * b], 0), "fork shadow stage");
                    PT_HIP(timed(c, prof, 3, s2, [&] { return launch_shadow(L.lds, count, grid, block, s2, c->view, wb, b, ovf2, L.gcap, xcd); }), "shadow");
                    PT_HIP(hipEventRecord(c->side_ev[2 * b + 1], s2), "join shadow stage");
                    pend = b;
                } else {
                    PT_HIP(timed(c, prof, 3, s, [&] { return launch_shadow(L.lds, count, grid, block, s, c->view, wb, b, ovf, L.gcap, xcd); }), "shadow");
                }
            }
        }
        if (pend >= 0) PT_HIP(hipStreamWaitEvent(s, c->side_ev[2 * pend + 1], 0), "join shadow stage");
        *Lbuf = wb.L;
        remember_frame(c, a, counts, w.ncounts, 1, acc != nullptr, promotes);
    }
    c->last_trav = trav;
    return PT_OK;
}

// the largest triangles' ids follow the light table in the light buffer
size_t hot_ids_offset(const pt_ctx* c) { return std::max<size_t>(1, c->bvh.lights.size()) * sizeof(LightEntry); }

// which shading features the scene uses (kAttrNormals | kAttrUV | kAttrCoat);
// nonzero selects the shading kernels' extended variant
int32_t shading_flags(const pt_ctx* c) {
    int32_t f = (c->attr_n.empty() ? 0 : kAttrNormals) | (c->attr_uv.empty() ? 0 : kAttrUV);
    for (size_t i = 0; i < c->mats.size(); i += 4)
        if ((int)c->mats[i] == PT_COATED) f |= kAttrCoat;
    return f;
}

SceneView make_view(const pt_ctx* c, const pt_scene_buffers* b) {
    SceneView v{};
    v.nodes = reinterpret_cast<const float4*>(b->nodes);
    v.tris = reinterpret_cast<const float4*>(b->tris);
    v.lights = reinterpret_cast<const LightEntry*>(b->lights);
    v.mats = reinterpret_cast<const float4*>(b->materials);
    v.albedo = b->albedo;
    v.emission = b->emission;
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
    v.hot_ids = reinterpret_cast<const uint32_t*>(static_cast<const char*>(b->lights) + hot_ids_offset(c));
    v.n_hot = (int32_t)c->bvh.hot_ids.size();
    v.insts = c->bvh.insts.empty() ? nullptr : reinterpret_cast<const float4*>(b->instances);
    v.n_inst = (int32_t)(c->bvh.insts.size() / kInstRecord);
    v.attrs = c->attr_leaf.empty() ? nullptr : reinterpret_cast<const float4*>(b->attributes);
    v.attr_flags = shading_flags(c);
    return v;
}

}  // namespace

extern "C" {

int32_t pt_version(void) { return 10000; }

const char* pt_last_error(void) { return g_err.c_str(); }

pt_status pt_create(pt_ctx** out, int32_t device) {
    if (!out) return fail(PT_EINVAL, "null output pointer");
    *out = nullptr;
    pt_ctx* c = new pt_ctx();
    if (device >= 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || n == 0) {
            delete c;
            return fail(PT_EHIP, std::string("no HIP device: ") + (e != hipSuccess ? hipGetErrorString(e) : "count is 0"));
        }
        if (device >= n) {
            delete c;
            return fail(PT_EHIP, "device index out of range");
        }
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, device);
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "hipGetDeviceProperties");
        }
        c->num_cu = prop.multiProcessorCount;
        c->lds_per_block = prop.sharedMemPerBlock;
        c->device = device;
        c->in_flight = frames_in_flight_for_queues();
        // the device address of this GPU's scratch array (the allocation-free
        // entry point's memory), looked up once per device
        e = noalloc_scratch_init(device);
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "device scratch address");
        }
    }
    *out = c;
    return PT_OK;
}

pt_status pt_destroy(pt_ctx* c) {
    if (!c) return PT_OK;
    if (c->device >= 0) {
        (void)hipSetDevice(c->device);
        for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
        if (c->aux_ready) {
            for (int i = 0; i < c->in_flight; ++i) {
                (void)hipStreamDestroy(c->aux[i]);
                (void)hipEventDestroy(c->ev_stage[i]);
                (void)hipEventDestroy(c->ev_acc[i]);
            }
            (void)hipEventDestroy(c->ev_entry);
        }
        for (hipEvent_t e : c->side_ev) (void)hipEventDestroy(e);
        if (c->side) (void)hipStreamDestroy(c->side);
    }
    delete c;
    return PT_OK;
}

pt_status pt_load_scene(pt_ctx* c, const pt_scene_desc* s) {
    if (!c || !s) return fail(PT_EINVAL, "null argument");
    if (s->nv < 0 || s->nt < 0 || s->nm < 1) return fail(PT_EINVAL, "need nv >= 0, nt >= 0, nm >= 1");
    if (s->nt > 0 && (!s->positions || !s->indices || !s->tri_material || !s->albedo || !s->emission))
        return fail(PT_EINVAL, "null scene array");
    if (!s->materials) return fail(PT_EINVAL, "null material table");
    if ((int64_t)s->nt > kMaxTris) return fail(PT_EINVAL, "too many triangles");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(s->sky[i])) return fail(PT_EINVAL, "non-finite sky");
    for (int64_t i = 0; i < 3 * (int64_t)s->nv; ++i)
        if (!std::isfinite(s->positions[i])) return fail(PT_EINVAL, "non-finite vertex position");
    for (int i = 0; i < s->nm; ++i) {
        const float* m = s->materials + 4 * i;
        int t = (int)m[0];
        if ((float)t != m[0] || t < PT_LAMBERT || t > PT_COATED) return fail(PT_EINVAL, "unknown material type");
        if (!(m[1] >= 0.f && m[1] <= 1.f)) return fail(PT_EINVAL, "roughness must be in [0, 1]");
        if ((t == PT_DIELECTRIC || t == PT_COATED) && !(m[2] > 0.f && std::isfinite(m[2]))) return fail(PT_EINVAL, "bad ior");
        if (!(m[3] >= 0.f && std::isfinite(m[3]))) return fail(PT_EINVAL, "checker frequency must be finite and >= 0");
    }
    c->nt = s->nt;
    c->nm = s->nm;
    c->tri_v.resize(9 * (size_t)s->nt);
    c->tri_mat.assign(s->tri_material, s->tri_material + s->nt);
    for (int32_t i = 0; i < s->nt; ++i) {
        for (int k = 0; k < 3; ++k) {
            int32_t vi = s->indices[3 * (size_t)i + k];
            if (vi < 0 || vi >= s->nv) return fail(PT_EINVAL, "vertex index out of range");
            for (int a = 0; a < 3; ++a) c->tri_v[9 * (size_t)i + 3 * k + a] = s->positions[3 * (size_t)vi + a];
        }
        if (c->tri_mat[i] < 0 || c->tri_mat[i] >= s->nm) return fail(PT_EINVAL, "material index out of range");
    }
    c->albedo.assign(s->albedo, s->albedo + 3 * (size_t)s->nt);
    c->emission.assign(s->emission, s->emission + 3 * (size_t)s->nt);
    for (float v : c->albedo)
        if (!std::isfinite(v)) return fail(PT_EINVAL, "non-finite albedo");
    for (float v : c->emission)
        if (!std::isfinite(v) || v < 0.f) return fail(PT_EINVAL, "emission must be finite and >= 0");
    c->mats.assign(s->materials, s->materials + 4 * (size_t)s->nm);
    std::memcpy(c->sky, s->sky, sizeof c->sky);
    c->inst = InstanceSet{};
    c->nv = s->nv;
    c->tri_idx.assign(s->indices, s->indices + 3 * (size_t)s->nt);
    c->attr_n.clear();
    c->attr_uv.clear();
    c->attr_leaf.clear();
    c->loaded = true;
    c->built = false;
    c->bound = false;
    return PT_OK;
}

pt_status pt_set_instances(pt_ctx* c, const pt_instances_desc* d) {
    if (!c) return fail(PT_EINVAL, "null context");
    if (!c->loaded) return fail(PT_ESTATE, "no scene loaded");
    InstanceSet is;
    if (d && d->n_instances > 0) {
        if (d->n_meshes < 1 || !d->mesh_first || !d->mesh_count || !d->inst_mesh || !d->o2w || !d->w2o)
            return fail(PT_EINVAL, "null instance array");
        if ((int64_t)d->n_instances > (int64_t)kLeafFirstMask) return fail(PT_EINVAL, "too many instances");
        std::vector<std::pair<int32_t, int32_t>> ranges;
        for (int m = 0; m < d->n_meshes; ++m) {
            const int32_t f = d->mesh_first[m], n = d->mesh_count[m];
            if (f < 0 || n < 0 || (int64_t)f + n > c->nt) return fail(PT_EINVAL, "mesh range out of range");
            if (n > 0) ranges.emplace_back(f, n);
        }
        std::sort(ranges.begin(), ranges.end());
        for (size_t k = 1; k < ranges.size(); ++k)
            if (ranges[k - 1].first + ranges[k - 1].second > ranges[k].first) return fail(PT_EINVAL, "mesh ranges overlap");
        for (int q = 0; q < d->n_instances; ++q) {
            if (d->inst_mesh[q] < 0 || d->inst_mesh[q] >= d->n_meshes) return fail(PT_EINVAL, "instance mesh out of range");
            for (int k = 0; k < 12; ++k)
                if (!std::isfinite(d->o2w[12 * (size_t)q + k]) || !std::isfinite(d->w2o[12 * (size_t)q + k]))
                    return fail(PT_EINVAL, "non-finite instance matrix");
        }
        is.mesh_first.assign(d->mesh_first, d->mesh_first + d->n_meshes);
        is.mesh_count.assign(d->mesh_count, d->mesh_count + d->n_meshes);
        is.inst_mesh.assign(d->inst_mesh, d->inst_mesh + d->n_instances);
        is.o2w.assign(d->o2w, d->o2w + 12 * (size_t)d->n_instances);
        is.w2o.assign(d->w2o, d->w2o + 12 * (size_t)d->n_instances);
    }
    c->inst = std::move(is);
    c->built = false;
    c->bound = false;
    return PT_OK;
}

pt_status pt_set_attributes(pt_ctx* c, const pt_attributes_desc* d) {
    if (!c) return fail(PT_EINVAL, "null context");
    if (!c->loaded) return fail(PT_ESTATE, "no scene loaded");
    std::vector<float> an, au;
    if (d && (d->normals || d->uvs)) {
        if (d->nv != c->nv) return fail(PT_EINVAL, "attribute count differs from the scene's vertex count");
        for (int64_t i = 0; d->normals && i < 3 * (int64_t)d->nv; ++i)
            if (!std::isfinite(d->normals[i])) return fail(PT_EINVAL, "non-finite vertex normal");
        for (int64_t i = 0; d->uvs && i < 2 * (int64_t)d->nv; ++i)
            if (!std::isfinite(d->uvs[i])) return fail(PT_EINVAL, "non-finite texture coordinate");
        if (d->normals) {
            an.resize(9 * (size_t)c->nt);
            for (size_t i = 0; i < (size_t)c->nt; ++i)
                for (int k = 0; k < 3; ++k)
                    for (int a = 0; a < 3; ++a) an[9 * i + 3 * k + a] = d->normals[3 * (size_t)c->tri_idx[3 * i + k] + a];
        }
        if (d->uvs) {
            au.resize(6 * (size_t)c->nt);
            for (size_t i = 0; i < (size_t)c->nt; ++i)
                for (int k = 0; k < 3; ++k)
                    for (int a = 0; a < 2; ++a) au[6 * i + 2 * k + a] = d->uvs[2 * (size_t)c->tri_idx[3 * i + k] + a];
        }
    }
    c->attr_n = std::move(an);
    c->attr_uv = std::move(au);
    c->attr_leaf.clear();
    c->built = false;
    c->bound = false;
    return PT_OK;
}

pt_status pt_build_bvh(pt_ctx* c, const pt_bvh_opts* o, pt_bvh_info* info) {
    if (!c) return fail(PT_EINVAL, "null context");
    if (!c->loaded) return fail(PT_ESTATE, "no scene loaded");
    int max_leaf = o && o->max_leaf > 0 ? o->max_leaf : 1;
    int threads = o ? o->threads : 0;
    if (max_leaf > kMaxLeaf) return fail(PT_EINVAL, "max_leaf must be <= 8");
    auto t0 = std::chrono::steady_clock::now();
    try {
        c->bvh = c->inst.inst_mesh.empty()
                     ? build_scene(c->tri_v, c->tri_mat, c->emission, max_leaf, threads)
                     : build_instanced(c->tri_v, c->tri_mat, c->emission, c->inst, max_leaf, threads);
    } catch (const std::exception& e) {
        return fail(PT_ENOMEM, std::string("BVH build failed: ") + e.what());
    }
    // attribute records in leaf order, keyed by each triangle record's input id
    c->attr_leaf.clear();
    if (!c->attr_n.empty() || !c->attr_uv.empty()) {
        const size_t n = (size_t)c->nt;
        c->attr_leaf.assign(kAttrRecord * n, make_float4(0.f, 0.f, 0.f, 0.f));
        for (size_t j = 0; j < n; ++j) {
            uint32_t id;
            std::memcpy(&id, &c->bvh.tris[3 * j].w, sizeof id);
            float nn[9] = {}, uv[6] = {};
            if (!c->attr_n.empty()) std::memcpy(nn, &c->attr_n[9 * (size_t)id], sizeof nn);
            if (!c->attr_uv.empty()) std::memcpy(uv, &c->attr_uv[6 * (size_t)id], sizeof uv);
            float4* r = &c->attr_leaf[kAttrRecord * j];
            r[0] = make_float4(nn[0], nn[1], nn[2], uv[0]);
            r[1] = make_float4(nn[3], nn[4], nn[5], uv[1]);
            r[2] = make_float4(nn[6], nn[7], nn[8], uv[2]);
            r[3] = make_float4(uv[3], uv[4], uv[5], 0.f);
        }
    }
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    c->built = true;
    c->bound = false;
    if (info) {
        info->node_count = (int64_t)c->bvh.nodes.size();
        info->node_bytes = (int64_t)(c->bvh.nodes.size() * sizeof(Node4));
        info->tri_bytes = (int64_t)(std::max<size_t>(1, c->bvh.tris.size()) * sizeof(float4));
        info->light_count = (int64_t)c->bvh.lights.size();
        info->light_bytes = (int64_t)(std::max<size_t>(1, c->bvh.lights.size()) * sizeof(LightEntry) +
                                      sizeof(LightEntry) * (size_t)((kHotTris + 3) / 4));
        info->material_bytes = (int64_t)(c->mats.size() * sizeof(float));
        info->instance_count = (int64_t)(c->bvh.insts.size() / kInstRecord);
        info->instance_bytes = (int64_t)(c->bvh.insts.size() * sizeof(float4));
        info->attribute_bytes = (int64_t)(c->attr_leaf.size() * sizeof(float4));
        info->depth = c->bvh.depth;
        info->stack_entries = c->bvh.stack_entries;
        info->build_seconds = secs;
    }
    return PT_OK;
}

pt_status pt_get_bvh(pt_ctx* c, void* nodes, void* tris, void* lights, void* materials) {
    if (!c) return fail(PT_EINVAL, "null context");
    if (!c->built) return fail(PT_ESTATE, "BVH not built");
    if (nodes) std::memcpy(nodes, c->bvh.nodes.data(), c->bvh.nodes.size() * sizeof(Node4));
    if (tris) std::memcpy(tris, c->bvh.tris.data(), 3 * (size_t)c->nt * sizeof(float4));
    if (lights) std::memcpy(lights, c->bvh.lights.data(), c->bvh.lights.size() * sizeof(LightEntry));
    if (materials) std::memcpy(materials, c->mats.data(), c->mats.size() * sizeof(float));
    return PT_OK;
}

pt_status pt_bind_scene(pt_ctx* c, const pt_scene_buffers* b, void* stream) {
    if (!c || !b) return fail(PT_EINVAL, "null argument");
    if (c->device < 0) return fail(PT_ESTATE, "host-only context cannot bind device buffers");
    if (!c->built) return fail(PT_ESTATE, "BVH not built (pt_build_bvh)");
    const void* ptrs[4] = {b->nodes, b->tris, b->lights, b->materials};
    for (const void* p : ptrs)
        if (!p || (reinterpret_cast<uintptr_t>(p) % kAlign) != 0) return fail(PT_EINVAL, "scene buffers must be non-null and 256-byte aligned");
    if (c->nt > 0 && (!b->albedo || !b->emission)) return fail(PT_EINVAL, "null albedo/emission");
    if (!c->bvh.insts.empty() && (!b->instances || (reinterpret_cast<uintptr_t>(b->instances) % kAlign) != 0))
        return fail(PT_EINVAL, "a two-level scene needs a 256-byte aligned instance buffer");
    if (!c->attr_leaf.empty() && (!b->attributes || (reinterpret_cast<uintptr_t>(b->attributes) % kAlign) != 0))
        return fail(PT_EINVAL, "vertex attributes need a 256-byte aligned attribute buffer");
    PT_HIP(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    PT_HIP(hipMemcpyAsync(b->nodes, c->bvh.nodes.data(), c->bvh.nodes.size() * sizeof(Node4), hipMemcpyHostToDevice, s), "upload nodes");
    if (!c->bvh.tris.empty())
        PT_HIP(hipMemcpyAsync(b->tris, c->bvh.tris.data(), c->bvh.tris.size() * sizeof(float4), hipMemcpyHostToDevice, s), "upload triangles");
    if (!c->bvh.lights.empty())
        PT_HIP(hipMemcpyAsync(b->lights, c->bvh.lights.data(), c->bvh.lights.size() * sizeof(LightEntry), hipMemcpyHostToDevice, s), "upload lights");
    if (!c->bvh.hot_ids.empty())
        PT_HIP(hipMemcpyAsync(static_cast<char*>(b->lights) + hot_ids_offset(c), c->bvh.hot_ids.data(),
                              c->bvh.hot_ids.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s),
               "upload hot triangle ids");
    PT_HIP(hipMemcpyAsync(b->materials, c->mats.data(), c->mats.size() * sizeof(float), hipMemcpyHostToDevice, s), "upload materials");
    if (!c->bvh.insts.empty())
        PT_HIP(hipMemcpyAsync(b->instances, c->bvh.insts.data(), c->bvh.insts.size() * sizeof(float4),
                              hipMemcpyHostToDevice, s),
               "upload instances");
    if (!c->attr_leaf.empty())
        PT_HIP(hipMemcpyAsync(b->attributes, c->attr_leaf.data(), c->attr_leaf.size() * sizeof(float4),
                              hipMemcpyHostToDevice, s),
               "upload vertex attributes");
    if (b->upload_params && c->nt > 0) {
        PT_HIP(hipMemcpyAsync(b->albedo, c->albedo.data(), c->albedo.size() * sizeof(float), hipMemcpyHostToDevice, s), "upload albedo");
        PT_HIP(hipMemcpyAsync(b->emission, c->emission.data(), c->emission.size() * sizeof(float), hipMemcpyHostToDevice, s), "upload emission");
    }
    // the host copies above are pageable: make sure they have been consumed
    PT_HIP(hipStreamSynchronize(s), "upload sync");
    c->view = make_view(c, b);
    c->bound = true;
    return PT_OK;
}

pt_status pt_set_camera(pt_ctx* c, const pt_camera* cam) {
    if (!c || !cam) return fail(PT_EINVAL, "null argument");
    if (cam->width < 1 || cam->height < 1 || cam->width > 65536 || cam->height > 65536)
        return fail(PT_EINVAL, "image size must be in [1, 65536]");
    if (!(cam->vfov_deg > 0.0 && cam->vfov_deg < 180.0)) return fail(PT_EINVAL, "vfov must be in (0, 180)");
    const double* e = cam->eye;
    const double* t = cam->target;
    const double* u = cam->up;
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(e[i]) || !std::isfinite(t[i]) || !std::isfinite(u[i])) return fail(PT_EINVAL, "non-finite camera");
    // binary64 basis, rounded once: F = unit(target - eye), R = unit(F x up)
    // scaled by tan(vfov / 2) * W / H, U = (R x F) scaled by tan(vfov / 2)
    double f[3] = {t[0] - e[0], t[1] - e[1], t[2] - e[2]};
    double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(fl > 0.0)) return fail(PT_EINVAL, "eye and target coincide");
    f[0] = f[0] / fl; f[1] = f[1] / fl; f[2] = f[2] / fl;
    double r[3] = {f[1] * u[2] - f[2] * u[1], f[2] * u[0] - f[0] * u[2], f[0] * u[1] - f[1] * u[0]};
    double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rl > 0.0)) return fail(PT_EINVAL, "up is parallel to the view direction");
    r[0] = r[0] / rl; r[1] = r[1] / rl; r[2] = r[2] / rl;
    double v[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    double th = std::tan(0.5 * (cam->vfov_deg * (3.14159265358979323846 / 180.0)));
    double asp = (double)cam->width / (double)cam->height;
    for (int i = 0; i < 3; ++i) {
        c->cam.E[i] = (float)e[i];
        c->cam.R[i] = (float)(r[i] * (th * asp));
        c->cam.U[i] = (float)(v[i] * th);
        c->cam.F[i] = (float)f[i];
    }
    c->cam.W = cam->width;
    c->cam.H = cam->height;
    c->cam_set = true;
    return PT_OK;
}

pt_status pt_workspace_size(pt_ctx* c, const pt_render_args* a, uint64_t* bytes) {
    if (!c || !a || !bytes) return fail(PT_EINVAL, "null argument");
    if (!c->built) return fail(PT_ESTATE, "BVH not built");
    if (!c->cam_set) return fail(PT_ESTATE, "camera not set");
    if (a->spp < 1 || a->max_depth < 0 || a->max_depth > 1000) return fail(PT_EINVAL, "bad spp or max_depth");
    Launch L;
    pt_status st = launch_config(c, a, L);
    if (st) return st;
    *bytes = layout(c, a, L).total;
    return PT_OK;
}

pt_status pt_backward_workspace_size(pt_ctx* c, const pt_render_args* a, uint64_t* bytes) {
    if (!c || !a || !bytes) return fail(PT_EINVAL, "null argument");
    if (!c->built) return fail(PT_ESTATE, "BVH not built");
    if (!c->cam_set) return fail(PT_ESTATE, "camera not set");
    if (a->spp < 1 || a->max_depth < 0 || a->max_depth > 1000) return fail(PT_EINVAL, "bad spp or max_depth");
    Launch L;
    pt_status st = launch_config(c, a, L);
    if (st) return st;
    *bytes = layout(c, a, L, true).total;
    return PT_OK;
}

pt_status pt_render_frame(pt_ctx* c, const pt_render_args* a, float* img, float* acc, void* ws, uint64_t ws_bytes,
                          void* stream) {
    pt_status st = check_args(c, a);
    if (st) return st;
    if (!img) return fail(PT_EINVAL, "null image");
    if (!ws) return fail(PT_EINVAL, "null workspace");
    if ((reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return fail(PT_EINVAL, "workspace must be 256-byte aligned");
    Launch L;
    st = launch_config(c, a, L);
    if (st) return st;
    WsLayout w = layout(c, a, L);
    if (ws_bytes < w.total) return fail(PT_ENOMEM, "workspace too small (pt_workspace_size)");
    PT_HIP(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const bool prof = (a->flags & PT_FLAG_PROFILE) != 0;
    c->timers.clear();
    c->event_next = 0;
    const float4* Lbuf = nullptr;
    hipStream_t s2 = nullptr;
    if (a->mode == PT_MODE_WAVE && !(a->flags & PT_FLAG_SERIAL_STAGES)) {
        st = side_stream(c, 2 * (a->max_depth + 1), s2);
        if (st) return st;
    }
    st = enqueue_stages(c, a, L, w, static_cast<char*>(ws), s, img, acc, prof, &Lbuf, nullptr, s2);
    if (st) return st;
    if (a->mode == PT_MODE_WAVE) {
        PathParams pp{a->spp, a->max_depth, a->nee ? 1 : 0, a->rr_start, a->seed, a->frame, a->job, a->sampler};
        PT_HIP(timed(c, prof, 4, s, [&] { return launch_accumulate(dim3(L.grid), dim3(L.block), s, c->cam, pp, Lbuf, img, acc); }), "accumulate");
    }
    return PT_OK;
}

pt_status pt_render_frame_noalloc(pt_ctx* c, const pt_render_args* a, float* img, float* acc, void* stream) {
    pt_status st = check_args(c, a);
    if (st) return st;
    if (!img) return fail(PT_EINVAL, "null image");
    if (a->mode != PT_MODE_MEGA) return fail(PT_EUNSUPPORTED, "pt_render_frame_noalloc renders with PT_MODE_MEGA only");
    if (a->flags & PT_FLAG_PROFILE) return fail(PT_EINVAL, "PT_FLAG_PROFILE creates events; not in pt_render_frame_noalloc");
    Launch L;
    st = launch_config(c, a, L);
    if (st) return st;
    const WsLayout w = layout(c, a, L);
    if (w.total > kNoAllocScratchBytes)
        return fail(PT_ENOMEM, "the frame needs " + std::to_string(w.total) + " bytes of device scratch, more than the " +
                                   std::to_string(kNoAllocScratchBytes) +
                                   " the library holds per GPU: lower grid_mult or block, or raise stack_lds");
    void* ptr = noalloc_scratch(c->device);
    if (!ptr) return fail(PT_ESTATE, "no device scratch address for this device");
    PT_HIP(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    c->timers.clear();
    c->event_next = 0;
    const float4* Lbuf = nullptr;
    return enqueue_stages(c, a, L, w, static_cast<char*>(ptr), s, img, acc, false, &Lbuf);
}

pt_status pt_frames_workspace_size(pt_ctx* c, const pt_render_args* a, uint64_t* bytes) {
    if (!c || !a || !bytes) return fail(PT_EINVAL, "null argument");
    if (!c->built) return fail(PT_ESTATE, "BVH not built");
    if (!c->cam_set) return fail(PT_ESTATE, "camera not set");
    if (a->spp < 1 || a->max_depth < 0 || a->max_depth > 1000) return fail(PT_EINVAL, "bad spp or max_depth");
    Launch L;
    pt_status st = launch_config(c, a, L);
    if (st) return st;
    *bytes = (uint64_t)c->in_flight * frame_slot_bytes(c, layout(c, a, L));
    return PT_OK;
}

pt_status pt_render_frames(pt_ctx* c, const pt_render_args* a, int32_t n_frames, float* img, float* acc, void* ws,
                           uint64_t ws_bytes, void* stream) {
    pt_status st = check_args(c, a);
    if (st) return st;
    if (n_frames < 1) return fail(PT_EINVAL, "n_frames must be >= 1");
    if ((uint64_t)a->frame + (uint64_t)n_frames > 0xFFFFFFFFull) return fail(PT_EINVAL, "frame index overflows");
    if (a->flags & PT_FLAG_PROFILE) return fail(PT_EINVAL, "PT_FLAG_PROFILE is per frame (pt_render_frame)");
    if (!img) return fail(PT_EINVAL, "null image");
    if (!ws) return fail(PT_EINVAL, "null workspace");
    if ((reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return fail(PT_EINVAL, "workspace must be 256-byte aligned");
    Launch L;
    st = launch_config(c, a, L);
    if (st) return st;
    const WsLayout w = layout(c, a, L);
    const size_t slot = frame_slot_bytes(c, w);
    const int nf = c->in_flight;
    if (ws_bytes < (uint64_t)nf * slot) return fail(PT_ENOMEM, "workspace too small (pt_frames_workspace_size)");
    PT_HIP(hipSetDevice(c->device), "hipSetDevice");
    if (!c->aux_ready) {
        for (int i = 0; i < nf; ++i) {
            PT_HIP(hipStreamCreateWithFlags(&c->aux[i], hipStreamNonBlocking), "create stream");
            PT_HIP(hipEventCreateWithFlags(&c->ev_stage[i], hipEventDisableTiming), "create event");
            PT_HIP(hipEventCreateWithFlags(&c->ev_acc[i], hipEventDisableTiming), "create event");
        }
        PT_HIP(hipEventCreateWithFlags(&c->ev_entry, hipEventDisableTiming), "create event");
        c->aux_ready = true;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    c->timers.clear();
    c->event_next = 0;
    // everything the caller enqueued before (scene, parameters, outputs)
    // precedes both internal streams
    PT_HIP(hipEventRecord(c->ev_entry, s), "record event");
    for (int i = 0; i < nf; ++i) PT_HIP(hipStreamWaitEvent(c->aux[i], c->ev_entry, 0), "stream wait");
    const uint32_t npix = (uint32_t)c->cam.W * (uint32_t)c->cam.H;
    for (int32_t f = 0; f < n_frames; ++f) {
        const int k = f % nf;
        char* base = static_cast<char*>(ws) + k * slot;
        float* frame_img = reinterpret_cast<float*>(base + w.total);
        pt_render_args af = *a;
        af.frame = a->frame + (uint32_t)f;
        // the slot's previous frame must have been accumulated
        PT_HIP(hipStreamWaitEvent(c->aux[k], c->ev_acc[k], 0), "stream wait");
        const float4* Lbuf = nullptr;
        st = enqueue_stages(c, &af, L, w, base, c->aux[k], frame_img, nullptr, false, &Lbuf);
        if (st) return st;
        PT_HIP(hipEventRecord(c->ev_stage[k], c->aux[k]), "record event");
        PT_HIP(hipStreamWaitEvent(s, c->ev_stage[k], 0), "stream wait");
        PathParams pp{af.spp, af.max_depth, af.nee ? 1 : 0, af.rr_start, af.seed, af.frame, af.job, af.sampler};
        if (a->mode == PT_MODE_WAVE) PT_HIP(launch_accumulate(dim3(L.grid), dim3(L.block), s, c->cam, pp, Lbuf, img, acc), "accumulate");
        else PT_HIP(launch_average(dim3(L.grid), dim3(L.block), s, frame_img, npix, af.frame, img, acc), "average");
        PT_HIP(hipEventRecord(c->ev_acc[k], s), "record event");
    }
    return PT_OK;
}

pt_status pt_render_backward(pt_ctx* c, const pt_render_args* a, const float* d_image, float* d_albedo,
                             float* d_emission, void* ws, uint64_t ws_bytes, void* stream) {
    pt_status st = check_args(c, a);
    if (st) return st;
    if (a->rr_start >= 0) return fail(PT_EINVAL, "the adjoint needs Russian roulette off (rr_start < 0)");
    if (c->view.n_inst > 0) return fail(PT_EUNSUPPORTED, "the adjoint takes flat scenes only");
    if (!d_image || !d_albedo || !d_emission) return fail(PT_EINVAL, "null gradient buffer");
    if (!ws) return fail(PT_EINVAL, "null workspace");
    if ((reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return fail(PT_EINVAL, "workspace must be 256-byte aligned");
    const bool keep = (a->flags & PT_FLAG_KEEP_HITS) != 0;
    Launch L;
    st = launch_config(c, a, L);
    if (st) return st;
    WsLayout w = layout(c, a, L, true);
    if (ws_bytes < w.total) return fail(PT_ENOMEM, "workspace too small (pt_backward_workspace_size)");
    PT_HIP(hipSetDevice(c->device), "hipSetDevice");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    uint32_t* counts = reinterpret_cast<uint32_t*>(base + w.counts);
    unsigned long long* trav = reinterpret_cast<unsigned long long*>(base + w.trav);
    uint2* ovf = reinterpret_cast<uint2*>(base + w.ovf);
    PathParams pp{a->spp, a->max_depth, a->nee ? 1 : 0, -1, a->seed, a->frame, a->job, a->sampler};
    const bool prof = (a->flags & PT_FLAG_PROFILE) != 0;
    c->timers.clear();
    c->event_next = 0;
    PT_HIP(launch_init_counts(s, counts, w.ncounts, 0u), "init counters");
    PT_HIP(launch_init_counts(s, reinterpret_cast<uint32_t*>(trav), kTravWords, 0u), "init work counters");
    unsigned long long* cursor = reinterpret_cast<unsigned long long*>(base + w.adj);
    const float4* Lpath = nullptr;
    const VertexRecs rec{keep ? reinterpret_cast<uint2*>(base + w.rec_hit) : nullptr,
                         keep ? reinterpret_cast<uint8_t*>(base + w.rec_vis) : nullptr,
                         (uint32_t)((size_t)c->cam.W * c->cam.H * a->spp)};
    if (a->mode == PT_MODE_WAVE) {
        // replay A by the wavefront stages (bit-identical per-path radiance;
        // the hybrid tail and the other wavefront options apply), which
        // leave each path's radiance in their per-path buffer; replay B
        // counts its rays in the block after the cursors
        PT_HIP(launch_init_counts(s, reinterpret_cast<uint32_t*>(cursor), 8, 0u), "init path cursors");
        hipStream_t s2 = nullptr;
        if (!(a->flags & PT_FLAG_SERIAL_STAGES)) {
            st = side_stream(c, 2 * (a->max_depth + 1), s2);
            if (st) return st;
        }
        st = enqueue_stages(c, a, L, w, base, s, nullptr, nullptr, prof, &Lpath, keep ? &rec : nullptr, s2);
        if (st) return st;
        counts = reinterpret_cast<uint32_t*>(base + w.adj) + 4;
    } else {
        float4* Lp = reinterpret_cast<float4*>(base + w.adj + kAlign);
        PT_HIP(launch_init_counts(s, reinterpret_cast<uint32_t*>(cursor), 4, 0u), "init path cursors");
        PT_HIP(timed(c, prof, 9, s, [&] {
                   return launch_adjoint_radiance(L.lds, dim3(L.grid), dim3(L.block), s, c->view, c->cam, pp, Lp,
                                                  cursor, ovf, L.gcap, counts, rec);
               }),
               "adjoint replay A");
        Lpath = Lp;
    }
    PT_HIP(timed(c, prof, 7, s, [&] {
               return launch_adjoint(L.lds, dim3(L.grid), dim3(L.block), s, c->view, c->cam, pp, d_image, Lpath, cursor,
                                     d_albedo, d_emission, ovf, L.gcap, counts, a->mode == PT_MODE_WAVE ? 1 : 0, rec);
           }),
           "adjoint replay B");
    remember_frame(c, a, counts, a->mode == PT_MODE_WAVE ? 4 : w.ncounts, 2, false);
    c->last_replay_wave = a->mode == PT_MODE_WAVE;
    c->last_keep_hits = keep;
    c->last_ovf_a = reinterpret_cast<uint32_t*>(base + w.counts) + (w.ncounts - 1);
    c->last_trav = trav;
    return PT_OK;
}

pt_status pt_frame_stats_get(pt_ctx* c, pt_frame_stats* out) {
    if (!c || !out) return fail(PT_EINVAL, "null argument");
    std::memset(out, 0, sizeof *out);
    if (!c->last_valid) return fail(PT_ESTATE, "no frame rendered");
    PT_HIP(hipSetDevice(c->device), "hipSetDevice");
    // frames in flight ran on the internal streams
    if (c->aux_ready)
        for (int i = 0; i < c->in_flight; ++i) PT_HIP(hipStreamSynchronize(c->aux[i]), "stream sync");
    if (c->side) PT_HIP(hipStreamSynchronize(c->side), "stream sync");
    for (const StageTimer& t : c->timers) {
        PT_HIP(hipEventSynchronize(t.b), "event sync");
        float ms = 0.f;
        PT_HIP(hipEventElapsedTime(&ms, t.a, t.b), "event time");
        out->stage_ms[t.stage] += (double)ms;
        out->launches[t.stage] += 1;
    }
    std::vector<uint32_t> h(c->last_ncounts);
    PT_HIP(hipMemcpy(h.data(), c->last_counts, h.size() * sizeof(uint32_t), hipMemcpyDeviceToHost), "read counters");
    unsigned long long tv[kTravWords / 2];
    PT_HIP(hipMemcpy(tv, c->last_trav, sizeof tv, hipMemcpyDeviceToHost), "read work counters");
    const uint64_t npix = c->last_npix, npaths = npix * (uint64_t)c->last_spp;
    const double img_bytes = 12.0 + (c->last_acc ? 24.0 : 0.0);  // image write (+ running average RMW)
    if (c->last_kind != 1) {
        // megakernel / adjoint: [0] extension rays, [1] shadow rays, [2] overflow
        out->extension_rays = h[0];
        out->shadow_rays = h[1];
        const int k = c->last_kind == 0 ? 5 : 7;
        out->stage_items[k] = (int64_t)npaths;
        out->node_visits[k] = (int64_t)tv[0];
        out->tri_tests[k] = (int64_t)tv[1];
        // path state lives in registers: the megakernel writes the image
        // (and updates the running average); the adjoint writes each path's
        // radiance in replay A (16 B) and reads it and its pixel's image
        // adjoint in replay B (16 + 12 B)
        out->stage_bytes[k] = c->last_kind == 0 ? (double)npix * img_bytes : 28.0 * (double)npaths;
        if (c->last_kind == 2 && !c->last_replay_wave) {
            out->stage_items[9] = (int64_t)npaths;
            out->stage_bytes[9] = 16.0 * (double)npaths;
        }
        if (c->last_kind == 2 && c->last_keep_hits) {
            // the records: 9 bytes per path vertex (one per extension ray),
            // written by replay A and read by replay B
            out->stage_bytes[7] += 9.0 * (double)h[0];
            out->stage_bytes[9] += 9.0 * (double)h[0];
        }
        if (h[2]) return fail(PT_EOVERFLOW, "traversal stack overflow");
        if (c->last_kind == 2 && c->last_replay_wave) {
            uint32_t fa = 0;
            PT_HIP(hipMemcpy(&fa, c->last_ovf_a, sizeof fa, hipMemcpyDeviceToHost), "read counters");
            if (fa) return fail(PT_EOVERFLOW, "traversal stack overflow");
        }
        return PT_OK;
    }
    const int D = c->last_D;
    const uint32_t* cnt = h.data();
    const uint32_t* shc = h.data() + D + 2;
    const uint32_t tail = c->last_compact ? c->last_tail : 0u;
    const int tail_bounce = c->last_compact ? c->last_tail_bounce : 0;
    // per queued path: raygen writes ray_o, ray_d, pst, L (64 B); extend
    // reads ray_o, ray_d, writes hit (48 B); shade reads ray_o, ray_d, pst,
    // hit, L (80 B) and writes 48 B per continuation and per shadow record;
    // shadow reads 48 B per record; the tail reads a shade record (80 B) and
    // writes the final L (16 B); the sort reads hit, writes the key, reads
    // the key, writes the permutation (28 B)
    out->stage_items[0] = (int64_t)npaths;
    out->stage_bytes[0] = 64.0 * (double)npaths;
    for (int b = 0; b <= D; ++b) {
        out->extension_rays += cnt[b];
        out->stage_items[1] += cnt[b];
        if (c->last_sort && cnt[b] >= c->last_sort_threshold) out->stage_items[6] += (int64_t)c->last_sort * cnt[b];
        if ((tail && cnt[b] < tail) || (tail_bounce > 0 && b >= tail_bounce)) {
            out->stage_items[8] += cnt[b];
        } else {
            out->stage_items[2] += cnt[b];
            out->stage_bytes[2] += 48.0 * ((double)cnt[b + 1] + (double)shc[b]);
        }
        if (b < D && c->last_nee) {
            out->shadow_rays += shc[b];
            out->stage_items[3] += shc[b];
        }
    }
    out->extension_rays += h[2 * D + 3];
    out->shadow_rays += h[2 * D + 4];
    out->node_visits[1] = (int64_t)tv[0];
    out->tri_tests[1] = (int64_t)tv[1];
    out->node_visits[3] = (int64_t)tv[2];
    out->tri_tests[3] = (int64_t)tv[3];
    out->node_visits[8] = (int64_t)tv[4];
    out->tri_tests[8] = (int64_t)tv[5];
    out->stage_bytes[1] = 48.0 * (double)out->stage_items[1];
    out->stage_bytes[2] += 80.0 * (double)out->stage_items[2];
    out->stage_bytes[3] = 48.0 * (double)out->stage_items[3];
    out->stage_bytes[6] = 28.0 * (double)out->stage_items[6];
    out->stage_bytes[8] = 96.0 * (double)out->stage_items[8];
    // promote launches of the two-slot count buffer: one word read, three
    // written (16 B)
    out->stage_items[10] = c->last_promotes;
    out->stage_bytes[10] = 16.0 * (double)c->last_promotes;
    out->stage_items[4] = (int64_t)npix;
    out->stage_bytes[4] = (double)npix * (16.0 * c->last_spp + img_bytes);
    if (h[c->last_ncounts - 1]) return fail(PT_EOVERFLOW, "traversal stack overflow");
    return PT_OK;
}

}  // extern "C"

namespace {

struct BatchPlan {
    std::vector<JobDesc> jobs;
    std::vector<int> members;  // caller's job index of each job of this pool
    uint64_t total = 0, total_pix = 0;
    int device = -1, num_cu = 256, stack_entries = 1;
    size_t lds_per_block = 160 * 1024;
    Launch L{};
    uint32_t capacity = 0;
    int iters_per_graph = 8, use_graph = 1;
    bool attr = false;  // some job's scene has vertex attributes
    // workspace offsets
    size_t o_jobs = 0, o_ctl = 0, o_rem = 0, o_ts = 0, o_pool = 0, o_L = 0, o_ovf = 0, total_bytes = 0;
};

// one pool: the jobs `members` of the caller's list, `capacity` path slots
pt_status plan_batch(const pt_job* jobs, const std::vector<int>& members, const pt_batch_opts* o, uint32_t capacity,
                     BatchPlan& P) {
    const int n = (int)members.size();
    P.members = members;
    P.jobs.resize(n);
    for (int j = 0; j < n; ++j) {
        const pt_job& jb = jobs[members[j]];
        pt_status st = check_args(jb.ctx, &jb.args);
        if (st) return st;
        if (!jb.image_out) return fail(PT_EINVAL, "null job image");
        if (jb.ctx->view.n_inst > 0) return fail(PT_EUNSUPPORTED, "the batched launch takes flat scenes only");
        if (P.device < 0) {
            P.device = jb.ctx->device;
            P.num_cu = jb.ctx->num_cu;
            P.lds_per_block = jb.ctx->lds_per_block;
        } else if (P.device != jb.ctx->device) {
            return fail(PT_EINVAL, "all jobs of a batch must be on one device");
        }
        JobDesc& d = P.jobs[j];
        d.sc = jb.ctx->view;
        P.attr = P.attr || d.sc.attr_flags != 0;
        d.cam = jb.ctx->cam;
        d.pp = PathParams{jb.args.spp, jb.args.max_depth, jb.args.nee ? 1 : 0, jb.args.rr_start, jb.args.seed,
                          jb.args.frame, jb.args.job, jb.args.sampler};
        d.img = jb.image_out;
        d.npaths = (uint32_t)((uint64_t)d.cam.W * d.cam.H * jb.args.spp);
        d.npix = (uint32_t)((uint64_t)d.cam.W * d.cam.H);
        d.base = (uint32_t)P.total;
        d.pix_base = (uint32_t)P.total_pix;
        P.total += d.npaths;
        P.total_pix += d.npix;
        if (P.total >= 0xFFFFFFFFull) return fail(PT_EINVAL, "a batch holds fewer than 2^32 - 1 paths");
        P.stack_entries = std::max(P.stack_entries, jb.ctx->bvh.stack_entries);
    }
    P.capacity = capacity;
    P.iters_per_graph = o->iters_per_graph > 0 ? o->iters_per_graph : 8;
    if (P.iters_per_graph % 2 || P.iters_per_graph > 256) return fail(PT_EINVAL, "iters_per_graph must be even and <= 256");
    P.use_graph = o->use_graph;
    pt_render_args la{};
    la.block = o->block;
    la.grid_mult = o->grid_mult;
    P.L.block = la.block > 0 ? la.block : kDefaultBlock;
    int mult = la.grid_mult > 0 ? la.grid_mult : kDefaultGridMult;
    if (P.L.block < 64 || P.L.block > 256 || (P.L.block % 64) != 0) return fail(PT_EINVAL, "block must be a multiple of 64 in [64, 256]");
    if (mult < 1 || mult > 64) return fail(PT_EINVAL, "grid_mult must be in [1, 64]");
    P.L.grid = P.num_cu * mult;
    pt_status sl = stack_lds_for(o->stack_lds, P.stack_entries, P.L.block, P.lds_per_block, P.L.lds);
    if (sl) return sl;
    P.L.gcap = std::max(0, P.stack_entries - P.L.lds);
    P.L.nlanes = (uint32_t)P.L.grid * (uint32_t)P.L.block;
    size_t off = 0;
    P.o_jobs = off; off = align_up(off + sizeof(JobDesc) * n);
    P.o_ctl = off; off = align_up(off + sizeof(BatchCtl));
    P.o_rem = off; off = align_up(off + sizeof(uint32_t) * n);
    P.o_ts = off; off = align_up(off + sizeof(uint64_t) * n);
    P.o_pool = off; off = align_up(off + sizeof(float4) * (size_t)P.capacity * 10);
    P.o_L = off; off = align_up(off + sizeof(float4) * std::max<uint64_t>(P.total, 1));
    P.o_ovf = off; off = align_up(off + sizeof(uint2) * (size_t)P.L.gcap * P.L.nlanes);
    P.total_bytes = off;
    return PT_OK;
}

// The caller's jobs split into `pools` pools of about equal path counts
// (largest job first into the least loaded pool), each with its share of
// the path slots and its own workspace slice at offs[k].
pt_status plan_pools(const pt_job* jobs, int32_t n, const pt_batch_opts* o, std::vector<BatchPlan>& G,
                     std::vector<size_t>& offs, size_t& total_bytes) {
    if (!jobs || n < 1) return fail(PT_EINVAL, "need at least one job");
    if (n > 255) return fail(PT_EINVAL, "at most 255 jobs per batch");
    pt_batch_opts def{0, 0, 0, 0, 0, 1, 0};
    if (!o) o = &def;
    const uint32_t capacity = o->pool_capacity ? o->pool_capacity : (1u << 21);
    if (capacity < 64 || capacity > (1u << 28)) return fail(PT_EINVAL, "pool_capacity must be in [64, 2^28]");
    const int K = o->pools > 0 ? o->pools : 1;
    if (K > kMaxPools) return fail(PT_EINVAL, "pools must be in [0, 4]");
    if (K > n) return fail(PT_EINVAL, "pools must not exceed the number of jobs");
    if (K > 1 && capacity / (uint32_t)K < 64) return fail(PT_EINVAL, "pool_capacity / pools must be at least 64");
    std::vector<uint64_t> size(n);
    for (int j = 0; j < n; ++j) {
        if (!jobs[j].ctx) return fail(PT_EINVAL, "null job context");
        size[j] = (uint64_t)jobs[j].ctx->cam.W * (uint64_t)jobs[j].ctx->cam.H * (uint64_t)std::max(jobs[j].args.spp, 0);
    }
    std::vector<int> order(n);
    for (int j = 0; j < n; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return size[a] > size[b]; });
    std::vector<std::vector<int>> members(K);
    std::vector<uint64_t> load(K, 0);
    for (int j : order) {
        int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        members[k].push_back(j);
        load[k] += size[j];
    }
    G.assign(K, BatchPlan{});
    offs.assign(K, 0);
    total_bytes = 0;
    const uint32_t cap_k = K == 1 ? capacity : (capacity / (uint32_t)K) & ~63u;
    for (int k = 0; k < K; ++k) {
        if (members[k].empty()) return fail(PT_EINVAL, "a pool would hold no job");
        std::sort(members[k].begin(), members[k].end());
        pt_status st = plan_batch(jobs, members[k], o, cap_k, G[k]);
        if (st) return st;
        offs[k] = total_bytes;
        total_bytes = align_up(total_bytes + G[k].total_bytes);
    }
    return PT_OK;
}

BatchBufs batch_bufs(const BatchPlan& P, char* base, int n) {
    BatchBufs bb{};
    bb.jobs = reinterpret_cast<JobDesc*>(base + P.o_jobs);
    bb.njobs = n;
    bb.capacity = P.capacity;
    bb.ctl = reinterpret_cast<BatchCtl*>(base + P.o_ctl);
    bb.remaining = reinterpret_cast<uint32_t*>(base + P.o_rem);
    bb.done_ts = reinterpret_cast<uint64_t*>(base + P.o_ts);
    float4* pool = reinterpret_cast<float4*>(base + P.o_pool);
    const size_t C = P.capacity;
    bb.ray_o[0] = pool + 0 * C; bb.ray_o[1] = pool + 1 * C;
    bb.ray_d[0] = pool + 2 * C; bb.ray_d[1] = pool + 3 * C;
    bb.pst[0] = pool + 4 * C; bb.pst[1] = pool + 5 * C;
    bb.hit = pool + 6 * C;
    bb.sh_o = pool + 7 * C; bb.sh_d = pool + 8 * C; bb.sh_c = pool + 9 * C;
    bb.L = reinterpret_cast<float4*>(base + P.o_L);
    return bb;
}

}  // namespace

extern "C" {

pt_status pt_batch_workspace_size(const pt_job* jobs, int32_t n, const pt_batch_opts* o, uint64_t* bytes) {
    if (!bytes) return fail(PT_EINVAL, "null output");
    std::vector<BatchPlan> G;
    std::vector<size_t> offs;
    size_t total = 0;
    pt_status st = plan_pools(jobs, n, o, G, offs, total);
    if (st) return st;
    *bytes = total;
    return PT_OK;
}

pt_status pt_render_batch(const pt_job* jobs, int32_t n, const pt_batch_opts* o, void* ws, uint64_t ws_bytes,
                          void* stream, double* job_ms, pt_batch_result* res) {
    std::vector<BatchPlan> G;
    std::vector<size_t> offs;
    size_t total = 0;
    pt_status st = plan_pools(jobs, n, o, G, offs, total);
    if (st) return st;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return fail(PT_EINVAL, "workspace must be non-null and 256-byte aligned");
    if (ws_bytes < total) return fail(PT_ENOMEM, "workspace too small (pt_batch_workspace_size)");
    const int K = (int)G.size();
    const int device = G[0].device;
    for (int k = 1; k < K; ++k)
        if (G[k].device != device) return fail(PT_EINVAL, "all jobs of a batch must be on one device");
    PT_HIP(hipSetDevice(device), "hipSetDevice");
    auto t0 = std::chrono::steady_clock::now();
    char* base = static_cast<char*>(ws);
    hipStream_t user = reinterpret_cast<hipStream_t>(stream);
    // one private non-blocking stream (default priority) per pool, ordered
    // after the caller's work; the pools run concurrently
    struct Pool {
        hipStream_t s = nullptr;
        hipEvent_t done = nullptr;  // the pool's last enqueued graph (or iterations) has run
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        BatchBufs bb{};
        BatchCtl ctl{};
        uint64_t iters = 0, cap_iters = 0;
        bool active = false;
    };
    struct Cleanup {
        std::vector<Pool> pools;
        hipEvent_t ev = nullptr;
        ~Cleanup() {
            // on an early error return no pool may still run on the caller's workspace
            for (Pool& p : pools)
                if (p.s) (void)hipStreamSynchronize(p.s);
            for (Pool& p : pools) {
                if (p.ge) (void)hipGraphExecDestroy(p.ge);
                if (p.g) (void)hipGraphDestroy(p.g);
                if (p.done) (void)hipEventDestroy(p.done);
                if (p.s) (void)hipStreamDestroy(p.s);
            }
            if (ev) (void)hipEventDestroy(ev);
        }
    } cl;
    cl.pools.resize(K);
    PT_HIP(hipEventCreateWithFlags(&cl.ev, hipEventDisableTiming), "create event");
    PT_HIP(hipEventRecord(cl.ev, user), "record");
    uint64_t launches = 0;
    for (int k = 0; k < K; ++k) {
        Pool& p = cl.pools[k];
        const BatchPlan& P = G[k];
        const int nk = (int)P.jobs.size();
        PT_HIP(hipStreamCreateWithFlags(&p.s, hipStreamNonBlocking), "create stream");
        PT_HIP(hipEventCreateWithFlags(&p.done, hipEventDisableTiming), "create event");
        PT_HIP(hipStreamWaitEvent(p.s, cl.ev, 0), "wait");
        char* pb = base + offs[k];
        p.bb = batch_bufs(P, pb, nk);
        PT_HIP(hipMemcpyAsync(p.bb.jobs, P.jobs.data(), sizeof(JobDesc) * nk, hipMemcpyHostToDevice, p.s), "upload jobs");
        PT_HIP(launch_batch_init(p.s, p.bb, (uint32_t)P.total), "batch init");
        // an upper bound on iterations: each iteration retires at least one
        // path vertex of the oldest path in the pool
        int max_depth = 0;
        for (const JobDesc& d : P.jobs) max_depth = std::max(max_depth, d.pp.D);
        p.cap_iters = (P.total / P.capacity + 2) * (uint64_t)(max_depth + 2) * 2 + 64;
        if (P.use_graph) {
            uint2* ovf = reinterpret_cast<uint2*>(pb + P.o_ovf);
            dim3 grid(P.L.grid), block(P.L.block);
            PT_HIP(hipStreamBeginCapture(p.s, hipStreamCaptureModeThreadLocal), "begin capture");
            hipError_t ce = hipSuccess;
            for (int it = 0; it < P.iters_per_graph && ce == hipSuccess; ++it)
                ce = launch_batch_iteration(P.L.lds, grid, block, p.s, p.bb, it & 1, ovf, P.L.gcap, P.attr);
            hipError_t ee = hipStreamEndCapture(p.s, &p.g);
            if (ce != hipSuccess) return hip_fail(ce, "capture launches");
            if (ee != hipSuccess) return hip_fail(ee, "end capture");
            PT_HIP(hipGraphInstantiate(&p.ge, p.g, nullptr, nullptr, 0), "instantiate graph");
        }
        p.active = true;
    }
    // enqueue the next graph (or two plain iterations) of pool k
    auto enqueue = [&](int k) -> pt_status {
        Pool& p = cl.pools[k];
        const BatchPlan& P = G[k];
        if (P.use_graph) {
            PT_HIP(hipGraphLaunch(p.ge, p.s), "graph launch");
            p.iters += P.iters_per_graph;
        } else {
            uint2* ovf = reinterpret_cast<uint2*>(base + offs[k] + P.o_ovf);
            for (int it = 0; it < 2; ++it)
                PT_HIP(launch_batch_iteration(P.L.lds, dim3(P.L.grid), dim3(P.L.block), p.s, p.bb, it & 1, ovf, P.L.gcap,
                                              P.attr),
                       "batch iteration");
            p.iters += 2;
        }
        ++launches;
        PT_HIP(hipEventRecord(p.done, p.s), "record");
        return PT_OK;
    };
    for (int k = 0; k < K; ++k) {
        st = enqueue(k);
        if (st) return st;
    }
    // Poll the pools: a pool whose work has run reads its control block and,
    // unless it has finished, gets its next graph at once, so each stream
    // stays busy while the others run.
    int nactive = K;
    while (nactive > 0) {
        bool progressed = false;
        for (int k = 0; k < K; ++k) {
            Pool& p = cl.pools[k];
            if (!p.active) continue;
            hipError_t q = hipEventQuery(p.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return hip_fail(q, "batch event");
            progressed = true;
            PT_HIP(hipMemcpyAsync(&p.ctl, p.bb.ctl, sizeof p.ctl, hipMemcpyDeviceToHost, p.s), "read control");
            PT_HIP(hipStreamSynchronize(p.s), "batch sync");
            if (p.ctl.err) return fail(PT_EOVERFLOW, "traversal stack overflow");
            if (p.ctl.done) {
                p.active = false;
                --nactive;
                continue;
            }
            if (p.iters > p.cap_iters) return fail(PT_EOVERFLOW, "batch did not finish within its iteration bound");
            st = enqueue(k);
            if (st) return st;
        }
        if (!progressed) std::this_thread::yield();
    }
    uint64_t t_start = ~0ull;
    int64_t iterations = 0;
    std::vector<std::vector<uint64_t>> ts(K);
    for (int k = 0; k < K; ++k) {
        Pool& p = cl.pools[k];
        const BatchPlan& P = G[k];
        PT_HIP(launch_batch_accumulate(dim3(P.L.grid), dim3(P.L.block), p.s, p.bb, (uint32_t)P.total_pix), "batch accumulate");
        ts[k].resize(P.jobs.size());
        PT_HIP(hipMemcpyAsync(ts[k].data(), p.bb.done_ts, sizeof(uint64_t) * P.jobs.size(), hipMemcpyDeviceToHost, p.s),
               "read timestamps");
        PT_HIP(hipStreamSynchronize(p.s), "batch final sync");
        t_start = std::min<uint64_t>(t_start, p.ctl.t_start);
        iterations += (int64_t)p.ctl.iterations;
    }
    // the caller's stream continues after every pool's work
    for (int k = 0; k < K; ++k) {
        PT_HIP(hipEventRecord(cl.pools[k].done, cl.pools[k].s), "record done");
        PT_HIP(hipStreamWaitEvent(user, cl.pools[k].done, 0), "caller waits");
    }
    if (job_ms) {
        int rate_khz = 0;
        PT_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device), "wall clock rate");
        for (int k = 0; k < K; ++k)
            for (size_t i = 0; i < G[k].members.size(); ++i) {
                const uint64_t t = ts[k][i];
                job_ms[G[k].members[i]] =
                    rate_khz > 0 && t >= t_start ? (double)(t - t_start) / (double)rate_khz : -1.0;
            }
    }
    if (res) {
        res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        uint64_t paths = 0;
        for (const BatchPlan& P : G) paths += P.total;
        res->path_samples = (int64_t)paths;
        res->iterations = iterations;
        res->launches = (int64_t)launches;
    }
    return PT_OK;
}

pt_status pt_sync(pt_ctx* c, void* stream) {
    if (!c) return fail(PT_EINVAL, "null context");
    if (c->device < 0) return PT_OK;
    PT_HIP(hipSetDevice(c->device), "hipSetDevice");
    PT_HIP(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)), "hipStreamSynchronize");
    return PT_OK;
}

}  // extern "C"
