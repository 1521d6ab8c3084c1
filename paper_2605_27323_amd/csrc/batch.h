// Batched wavefront over many jobs (scenes, cameras, resolutions, spp) that
// share one pool of path slots.  Every iteration: a scheduler refills the
// free slots from a global cursor over all jobs' paths (path regeneration),
// then extend / shade / shadow run over the whole pool.  A path's state
// carries its job and its vertex index, so paths of different jobs and
// depths share the queues.  Shared by the HIP kernels and the CPU emulator.
#pragma once
#include "wavefront.h"

namespace ptmi {

struct JobDesc {
    SceneView sc;
    CamView cam;
    PathParams pp;
    float* img;
    uint32_t base;    // first global path index of the job
    uint32_t npaths;  // W * H * spp
    uint32_t pix_base;  // first global pixel index of the job
    uint32_t npix;
};

// pool control block (device memory, one per batch)
struct BatchCtl {
    uint32_t total;        // paths over all jobs
    uint32_t cursor;       // next path to start
    uint32_t live[2];      // paths in queue q after compaction
    uint32_t count;        // paths in the current queue (live + regenerated)
    uint32_t regen_first;  // first slot refilled this iteration
    uint32_t regen_n;      // slots refilled this iteration
    uint32_t regen_path;   // first path id refilled this iteration
    uint32_t shadow;       // shadow records this iteration
    uint32_t done;         // all paths finished
    uint32_t iterations;
    uint32_t err;
    uint64_t t_start;      // device wall clock at the first iteration
};

struct BatchBufs {
    JobDesc* jobs;
    int32_t njobs;
    uint32_t capacity;
    BatchCtl* ctl;
    uint32_t* remaining;  // [njobs] paths not finished
    uint64_t* done_ts;    // [njobs] device wall clock when the job's last path finished
    float4* ray_o[2];     // (origin, global path id)
    float4* ray_d[2];     // (direction, last pdf)
    float4* pst[2];       // (throughput, meta: vertex k | smooth << 16 | job << 24)
    float4* hit;
    float4* sh_o;
    float4* sh_d;
    float4* sh_c;
    float4* L;            // [total] by global path id
};

PT_DEV uint32_t meta_pack(uint32_t k, uint32_t smooth, uint32_t job) { return k | (smooth << 16) | (job << 24); }

PT_DEV int find_job(const BatchBufs& bb, uint32_t g) {
    int lo = 0, hi = bb.njobs - 1;  // last job with base <= g
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (bb.jobs[mid].base <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// scheduler (one lane): refill free slots of queue q from the cursor
PT_DEV void batch_schedule(const BatchBufs& bb, int q) {
    BatchCtl& c = *bb.ctl;
    const uint32_t live = c.live[q];
    const uint32_t room = bb.capacity - live;
    const uint32_t left = c.total - c.cursor;
    const uint32_t take = room < left ? room : left;
    c.regen_first = live;
    c.regen_n = take;
    c.regen_path = c.cursor;
    c.cursor += take;
    c.count = live + take;
    c.live[q ^ 1] = 0u;
    c.shadow = 0u;
    if (c.count == 0u) c.done = 1u;
    else c.iterations += 1u;
}

// new path in slot (regen_first + i) of queue q
PT_DEV void batch_regen_item(const BatchBufs& bb, int q, uint32_t i) {
    const BatchCtl& c = *bb.ctl;
    const uint32_t slot = c.regen_first + i;
    const uint32_t g = c.regen_path + i;
    const int j = find_job(bb, g);
    const JobDesc& jd = bb.jobs[j];
    const uint32_t local = g - jd.base;
    const uint32_t pix = local / (uint32_t)jd.pp.spp;
    const uint32_t s = local - pix * (uint32_t)jd.pp.spp;
    const uint32_t sample = jd.pp.frame * (uint32_t)jd.pp.spp + s;
    f3 o, d;
    camera_sample(jd.cam, jd.pp, pix, sample, o, d);
    bb.ray_o[q][slot] = make_float4(o.x, o.y, o.z, u2f(g));
    bb.ray_d[q][slot] = make_float4(d.x, d.y, d.z, 0.f);
    bb.pst[q][slot] = make_float4(1.f, 1.f, 1.f, u2f(meta_pack(1u, 0u, (uint32_t)j)));
    bb.L[g] = make_float4(0.f, 0.f, 0.f, 0.f);
}

template <int LDS, bool COUNT = false>
PT_DEV void batch_extend_item(const BatchBufs& bb, int q, uint32_t i, TravStack<LDS, COUNT>& st) {
    const float4 o4 = bb.ray_o[q][i], d4 = bb.ray_d[q][i];
    const uint32_t job = f2u(bb.pst[q][i].w) >> 24;
    const SceneView& sc = bb.jobs[job].sc;
    Ray ray = make_ray(xyz(o4), xyz(d4));
    Hit h = closest_hit<LDS>(sc, ray, INFINITY, st);
    bb.hit[i] = make_float4(h.t, 0.f, 0.f, u2f(h.tri));
}

// shade slot i of queue q; returns true if the path finished here (the
// caller decrements its job's counter); vo / sh / ps / meta describe what
// to enqueue.  ATTR: some job's scene has vertex attributes.
template <bool ATTR = false>
PT_DEV bool batch_shade_item(const BatchBufs& bb, int q, uint32_t i, VertexOut& vo, ShadowReq& sh, PathState& ps,
                             uint32_t& g, uint32_t& meta) {
    const float4 o4 = bb.ray_o[q][i], d4 = bb.ray_d[q][i], p4 = bb.pst[q][i], h4 = bb.hit[i];
    g = f2u(o4.w);
    const uint32_t m = f2u(p4.w);
    const uint32_t k = m & 0xFFFFu, job = m >> 24;
    const JobDesc& jd = bb.jobs[job];
    const uint32_t local = g - jd.base;
    const uint32_t pix = local / (uint32_t)jd.pp.spp;
    const uint32_t s = local - pix * (uint32_t)jd.pp.spp;
    const uint32_t sample = jd.pp.frame * (uint32_t)jd.pp.spp + s;
    ps.beta = xyz(p4);
    ps.L = mk3(0.f, 0.f, 0.f);
    ps.p_prev = d4.w;
    ps.prev_smooth = (int)((m >> 16) & 1u);
    Hit h;
    h.t = h4.x;
    h.tri = f2u(h4.w);
    h.id = 0;
    hit_barycentrics(jd.sc, xyz(o4), xyz(d4), h);
    vo = shade_vertex<false, ATTR>(jd.sc, jd.pp, pix, sample, (int)k, xyz(d4), h, ps, sh);
    if (vo.addL) {  // the radiance is read only where this vertex adds to it
        ps.L = xyz(bb.L[g]);
        add_radiance(ps, vo);
        bb.L[g] = make_float4(ps.L.x, ps.L.y, ps.L.z, 0.f);
    }
    meta = meta_pack(k + 1u, (uint32_t)ps.prev_smooth, job);
    // a path with a pending light sample finishes after the shadow stage;
    // its job counter is decremented there
    return !vo.cont && !sh.valid;
}

PT_DEV void batch_write_continuation(const BatchBufs& bb, int q, uint32_t j, const VertexOut& vo, const PathState& ps,
                                     uint32_t g, uint32_t meta) {
    bb.ray_o[q][j] = make_float4(vo.o.x, vo.o.y, vo.o.z, u2f(g));
    bb.ray_d[q][j] = make_float4(vo.d.x, vo.d.y, vo.d.z, ps.p_prev);
    bb.pst[q][j] = make_float4(ps.beta.x, ps.beta.y, ps.beta.z, u2f(meta));
}

// shadow record j: (origin, global path id), (direction, job | last << 31), beta*C
PT_DEV void batch_write_shadow(const BatchBufs& bb, uint32_t j, const ShadowReq& sh, uint32_t g, uint32_t job,
                               bool last) {
    bb.sh_o[j] = make_float4(sh.o.x, sh.o.y, sh.o.z, u2f(g));
    bb.sh_d[j] = make_float4(sh.d.x, sh.d.y, sh.d.z, u2f(job | (last ? 0x80000000u : 0u)));
    bb.sh_c[j] = make_float4(sh.contrib.x, sh.contrib.y, sh.contrib.z, 0.f);
}

// unoccluded shadow record i: add its beta * C to its path
PT_DEV void batch_shadow_add(const BatchBufs& bb, uint32_t i) {
    const uint32_t g = f2u(bb.sh_o[i].w);
    const float4 c4 = bb.sh_c[i];
    const float4 l4 = bb.L[g];
    bb.L[g] = make_float4(l4.x + c4.x, l4.y + c4.y, l4.z + c4.z, 0.f);
}

// shadow record i: returns true if it ends its path (caller decrements the
// job counter) and sets job
template <int LDS, bool COUNT = false>
PT_DEV bool batch_shadow_item(const BatchBufs& bb, uint32_t i, TravStack<LDS, COUNT>& st, uint32_t& job) {
    const float4 o4 = bb.sh_o[i], d4 = bb.sh_d[i];
    const uint32_t tag = f2u(d4.w);
    job = tag & 0x7FFFFFFFu;
    Ray ray = make_ray(xyz(o4), xyz(d4));
    if (!any_hit<LDS>(bb.jobs[job].sc, ray, kShadowTmax, st)) batch_shadow_add(bb, i);
    return (tag >> 31) != 0u;
}

// global pixel index -> (job, pixel): mean over the pixel's spp paths
PT_DEV void batch_accumulate_item(const BatchBufs& bb, uint32_t gp) {
    int lo = 0, hi = bb.njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (bb.jobs[mid].pix_base <= gp) lo = mid;
        else hi = mid - 1;
    }
    const JobDesc& jd = bb.jobs[lo];
    const uint32_t pix = gp - jd.pix_base;
    accumulate_item(jd.pp, bb.L + jd.base, jd.img, nullptr, pix);
}

}  // namespace ptmi
