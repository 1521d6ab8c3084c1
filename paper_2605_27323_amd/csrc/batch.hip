// Batched persistent wavefront kernels (see batch.h): one pool of path
// slots shared by many jobs, refilled from a global cursor every iteration.
// The host captures a fixed number of iterations into a hipGraph and replays
// it until the device control block reports that every path has finished.
#include "batch.h"
#include "wave.h"

namespace ptmi {

namespace {

template <int LDS>
__device__ __forceinline__ TravStack<LDS> stack_b(uint32_t* smem, uint2* ovf, int gcap) {
    return make_trav_stack<LDS>(reinterpret_cast<uint2*>(smem) + threadIdx.x, (int)blockDim.x, ovf,
                                blockIdx.x * blockDim.x + threadIdx.x, (int)(gridDim.x * blockDim.x), gcap);
}

// wave-aggregated job counters: every lane of the wave calls this; lanes
// with fin set retire one path of job `job`.  One atomic per distinct job in
// the wave (usually one) instead of one per path; the lane whose
// subtraction reaches zero stamps the job's completion time.
__device__ __forceinline__ void jobs_finished(const BatchBufs& bb, bool fin, uint32_t job) {
    uint64_t m = __ballot(fin);
    while (m) {
        const int leader = __ffsll((unsigned long long)m) - 1;
        const uint32_t j0 = __shfl(job, leader);
        const uint64_t same = __ballot(fin && job == j0);
        if ((int)lane_id() == leader) {
            const uint32_t n = (uint32_t)__popcll(same);
            if (atomicSub(&bb.remaining[j0], n) == n) bb.done_ts[j0] = wall_clock64();
        }
        m &= ~same;
    }
}

}  // namespace

__global__ void k_batch_init(BatchBufs bb, uint32_t total) {
    const int t = threadIdx.x;
    if (t == 0) {
        BatchCtl& c = *bb.ctl;
        c.total = total;
        c.cursor = 0u;
        c.live[0] = c.live[1] = 0u;
        c.count = c.regen_first = c.regen_n = c.regen_path = c.shadow = 0u;
        c.done = 0u;
        c.iterations = 0u;
        c.err = 0u;
        c.t_start = wall_clock64();
    }
    for (int j = t; j < bb.njobs; j += blockDim.x) {
        bb.remaining[j] = bb.jobs[j].npaths;
        bb.done_ts[j] = 0ull;
    }
}

__global__ void k_batch_sched(BatchBufs bb, int q) {
    if (threadIdx.x == 0 && blockIdx.x == 0) batch_schedule(bb, q);
}

__global__ void __launch_bounds__(256) k_batch_regen(BatchBufs bb, int q) {
    const uint32_t n = bb.ctl->regen_n;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        batch_regen_item(bb, q, i);
}

// persistent traversal over the pool (see k_extend): each wave owns a chunk
// of the queue and refills finished lanes from it; a lane's scene is its
// path's job's scene
template <int LDS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_batch_extend(BatchBufs bb, int q, uint2* __restrict__ ovf, int gcap) {
    extern __shared__ __align__(8) uint32_t smem[];
    TravStack<LDS> st = stack_b<LDS>(smem, ovf, gcap);
    uint32_t next, end;
    wave_chunk(bb.ctl->count, next, end);
    bool live = false;
    uint32_t item = 0, ref = 0;
    SceneView sc{};
    Ray ray;
    Hit h;
    while (true) {
        const uint64_t idle = __ballot(!live);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (next < end && (nidle >= kRefill || nidle == 64u)) {
            if (!live) {
                const uint32_t i = next + rank_in(idle);
                if (i < end) {
                    const float4 o4 = bb.ray_o[q][i], d4 = bb.ray_d[q][i];
                    sc = bb.jobs[f2u(bb.pst[q][i].w) >> 24].sc;
                    ray = make_ray(xyz(o4), xyz(d4));
                    closest_begin<LDS>(INFINITY, h, ref, st);
                    item = i;
                    live = true;
                }
            }
            next = min(next + nidle, end);
        }
        if (__ballot(live) == 0ull) {
            if (next < end) continue;
            break;
        }
        if (live && !closest_step<LDS>(sc, ray, INFINITY, h, ref, st)) {
            bb.hit[item] = make_float4(h.t, 0.f, 0.f, u2f(h.tri));
            live = false;
        }
    }
    if (st.overflow) atomicOr(&bb.ctl->err, 1u);
}

// slots of the next queue and of the shadow queue reserved once per block
// and trip (see k_shade)
// four waves per SIMD, as k_shade (without attributes: 128 VGPRs, no spill)
template <bool ATTR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_batch_shade(BatchBufs bb, int q) {
    const uint32_t nlanes = gridDim.x * blockDim.x;
    const uint32_t count = bb.ctl->count;
    __shared__ BlockReserve br;
    int par = 0;
    for (uint32_t bbase = blockIdx.x * blockDim.x; bbase < count; bbase += nlanes, par ^= 1) {
        const uint32_t i = bbase + threadIdx.x;
        VertexOut vo;
        ShadowReq sh;
        PathState ps;
        vo.cont = false;
        sh.valid = false;
        uint32_t g = 0, meta = 0;
        bool finished = false;
        if (i < count) finished = batch_shade_item<ATTR>(bb, q, i, vo, sh, ps, g, meta);
        jobs_finished(bb, finished, meta >> 24);
        const uint64_t mk = __ballot(vo.cont), ms = __ballot(sh.valid);
        uint32_t jc, js;
        block_reserve2(br, par, &bb.ctl->live[q ^ 1], mk, &bb.ctl->shadow, ms, jc, js);
        if (vo.cont) batch_write_continuation(bb, q ^ 1, jc, vo, ps, g, meta);
        if (sh.valid) batch_write_shadow(bb, js, sh, g, meta >> 24, !vo.cont);
    }
}

// persistent any-hit over the shadow records; the job counters are updated
// every trip for the lanes whose record ended its path
template <int LDS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
k_batch_shadow(BatchBufs bb, uint2* __restrict__ ovf, int gcap) {
    extern __shared__ __align__(8) uint32_t smem[];
    TravStack<LDS> st = stack_b<LDS>(smem, ovf, gcap);
    uint32_t next, end;
    wave_chunk(bb.ctl->shadow, next, end);
    bool live = false;
    uint32_t item = 0, ref = 0, tag = 0;
    SceneView sc{};
    Ray ray;
    while (true) {
        const uint64_t idle = __ballot(!live);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (next < end && (nidle >= kRefill || nidle == 64u)) {
            if (!live) {
                const uint32_t i = next + rank_in(idle);
                if (i < end) {
                    const float4 o4 = bb.sh_o[i], d4 = bb.sh_d[i];
                    tag = f2u(d4.w);
                    sc = bb.jobs[tag & 0x7FFFFFFFu].sc;
                    ray = make_ray(xyz(o4), xyz(d4));
                    any_begin<LDS>(ref, st);
                    item = i;
                    live = true;
                }
            }
            next = min(next + nidle, end);
        }
        if (__ballot(live) == 0ull) {
            if (next < end) continue;
            break;
        }
        bool fin = false;
        if (live) {
            bool occluded = false;
            if (!any_step<LDS>(sc, ray, kShadowTmax, ref, st, occluded)) {
                live = false;
                if (!occluded) batch_shadow_add(bb, item);
                fin = (tag >> 31) != 0u;
            }
        }
        jobs_finished(bb, fin, tag & 0x7FFFFFFFu);
    }
    if (st.overflow) atomicOr(&bb.ctl->err, 1u);
}

__global__ void __launch_bounds__(256) k_batch_accumulate(BatchBufs bb, uint32_t total_pix) {
    for (uint32_t gp = blockIdx.x * blockDim.x + threadIdx.x; gp < total_pix; gp += gridDim.x * blockDim.x)
        batch_accumulate_item(bb, gp);
}

hipError_t launch_batch_init(hipStream_t s, const BatchBufs& bb, uint32_t total) {
    hipLaunchKernelGGL(k_batch_init, dim3(1), dim3(256), 0, s, bb, total);
    return hipGetLastError();
}

// one iteration of the pool on queue parity q
hipError_t launch_batch_iteration(int lds, dim3 grid, dim3 block, hipStream_t s, const BatchBufs& bb, int q,
                                  uint2* ovf, int gcap, bool attr) {
    const size_t sm = trav_stack_lds_bytes(lds, (int)block.x);
    hipLaunchKernelGGL(k_batch_sched, dim3(1), dim3(64), 0, s, bb, q);
    hipLaunchKernelGGL(k_batch_regen, grid, block, 0, s, bb, q);
#define X(N)                                                                              \
    if (lds == N) {                                                                       \
        hipLaunchKernelGGL(k_batch_extend<N>, grid, block, sm, s, bb, q, ovf, gcap);      \
        if (attr)                                                                         \
            hipLaunchKernelGGL(k_batch_shade<true>, grid, block, 0, s, bb, q);            \
        else                                                                              \
            hipLaunchKernelGGL(k_batch_shade<false>, grid, block, 0, s, bb, q);           \
        hipLaunchKernelGGL(k_batch_shadow<N>, grid, block, sm, s, bb, ovf, gcap);         \
        return hipGetLastError();                                                         \
    }
    X(8) X(16) X(24) X(32)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_batch_accumulate(dim3 grid, dim3 block, hipStream_t s, const BatchBufs& bb, uint32_t total_pix) {
    hipLaunchKernelGGL(k_batch_accumulate, grid, block, 0, s, bb, total_pix);
    return hipGetLastError();
}

}  // namespace ptmi
