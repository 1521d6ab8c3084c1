// Batched persistent wavefront kernels (see batch.h): one pool of path
// slots shared by many jobs, refilled from a global cursor every iteration.
// The host captures a fixed number of iterations into a hipGraph and replays
// it until the device control block reports that every path has finished.
#include "batch.h"

namespace ptmi {

namespace {

__device__ __forceinline__ uint32_t lane_id_b() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint32_t reserve_b(uint32_t* ctr, uint64_t m) {
    uint32_t base = 0;
    if (lane_id_b() == 0) base = atomicAdd(ctr, (uint32_t)__popcll(m));
    base = __builtin_amdgcn_readfirstlane(base);
    return base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <int LDS>
__device__ __forceinline__ TravStack<LDS> stack_b(uint32_t* smem, uint2* ovf, int gcap) {
    return make_trav_stack<LDS>(reinterpret_cast<uint2*>(smem) + threadIdx.x, (int)blockDim.x,
                                ovf + blockIdx.x * blockDim.x + threadIdx.x, (int)(gridDim.x * blockDim.x), gcap);
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
        if ((int)lane_id_b() == leader) {
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

template <int LDS>
__global__ void __launch_bounds__(256) k_batch_extend(BatchBufs bb, int q, uint2* __restrict__ ovf, int gcap) {
    extern __shared__ __align__(8) uint32_t smem[];
    TravStack<LDS> st = stack_b<LDS>(smem, ovf, gcap);
    const uint32_t count = bb.ctl->count;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        batch_extend_item<LDS>(bb, q, i, st);
    if (st.overflow) atomicOr(&bb.ctl->err, 1u);
}

__global__ void __launch_bounds__(256) k_batch_shade(BatchBufs bb, int q) {
    const uint32_t nlanes = gridDim.x * blockDim.x;
    const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t count = bb.ctl->count;
    for (uint32_t base = gtid & ~63u; base < count; base += nlanes) {
        const uint32_t i = base + (gtid & 63u);
        VertexOut vo;
        ShadowReq sh;
        PathState ps;
        vo.cont = false;
        sh.valid = false;
        uint32_t g = 0, meta = 0;
        bool finished = false;
        if (i < count) finished = batch_shade_item(bb, q, i, vo, sh, ps, g, meta);
        jobs_finished(bb, finished, meta >> 24);
        const uint64_t mk = __ballot(vo.cont);
        if (mk) {
            const uint32_t j = reserve_b(&bb.ctl->live[q ^ 1], mk);
            if (vo.cont) batch_write_continuation(bb, q ^ 1, j, vo, ps, g, meta);
        }
        const uint64_t ms = __ballot(sh.valid);
        if (ms) {
            const uint32_t j = reserve_b(&bb.ctl->shadow, ms);
            if (sh.valid) batch_write_shadow(bb, j, sh, g, meta >> 24, !vo.cont);
        }
    }
}

template <int LDS>
__global__ void __launch_bounds__(256) k_batch_shadow(BatchBufs bb, uint2* __restrict__ ovf, int gcap) {
    extern __shared__ __align__(8) uint32_t smem[];
    TravStack<LDS> st = stack_b<LDS>(smem, ovf, gcap);
    const uint32_t count = bb.ctl->shadow;
    const uint32_t nlanes = gridDim.x * blockDim.x;
    const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
    // wave-uniform trip count so that the job counters can be aggregated
    for (uint32_t base = gtid & ~63u; base < count; base += nlanes) {
        const uint32_t i = base + (gtid & 63u);
        uint32_t job = 0;
        bool fin = false;
        if (i < count) fin = batch_shadow_item<LDS>(bb, i, st, job);
        jobs_finished(bb, fin, job);
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
                                  uint2* ovf, int gcap) {
    const size_t sm = (size_t)lds * 2 * sizeof(uint32_t) * block.x;
    hipLaunchKernelGGL(k_batch_sched, dim3(1), dim3(64), 0, s, bb, q);
    hipLaunchKernelGGL(k_batch_regen, grid, block, 0, s, bb, q);
#define X(N)                                                                              \
    if (lds == N) {                                                                       \
        hipLaunchKernelGGL(k_batch_extend<N>, grid, block, sm, s, bb, q, ovf, gcap);      \
        hipLaunchKernelGGL(k_batch_shade, grid, block, 0, s, bb, q);                      \
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
