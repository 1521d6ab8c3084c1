// Render kernels of libptmi: the megakernel (paper Sec. 2.2: one thread per
// pixel traces its paths to the end) and the wavefront stages (Sec. 2.3 and
// 3.1: raygen, extend, shade, shadow, accumulate over structure-of-arrays
// path state, live paths compacted into a queue after every bounce).
#include "wavefront.h"
#include "wave.h"

namespace ptmi {

namespace {

template <int LDS, bool COUNT>
__device__ __forceinline__ TravStack<LDS, COUNT> make_stack(uint32_t* smem, uint2* ovf, int gcap, uint32_t gtid,
                                                            uint32_t nlanes) {
    return make_trav_stack<LDS, COUNT>(reinterpret_cast<uint2*>(smem) + threadIdx.x, (int)blockDim.x, ovf, gtid,
                                       (int)nlanes, gcap);
}

// Stage the light table (CDF words, leaf-order and input triangle indices)
// in the block's LDS so that the light choice is a binary search in LDS.
// Every thread of the block must call this (it synchronises the block).
__device__ __forceinline__ LightCache stage_lights(const SceneView& sc, uint32_t* buf) {
    if (sc.nl <= 0 || sc.nl > kLdsLights) return no_light_cache();
    for (int j = threadIdx.x; j < sc.nl; j += blockDim.x) {
        const LightEntry e = sc.lights[j];
        buf[j] = e.cdf;
        buf[kLdsLights + j] = e.tri;
        buf[2 * kLdsLights + j] = e.id;
    }
    __syncthreads();
    LightCache lc;
    lc.cdf = (const lds_u32*)buf;
    lc.tri = (const lds_u32*)(buf + kLdsLights);
    lc.id = (const lds_u32*)(buf + 2 * kLdsLights);
    lc.n = sc.nl;
    return lc;
}

}  // namespace

// ---------------------------------------------------------------------------
// megakernel
// ---------------------------------------------------------------------------
// pixels a wave takes from the frame's cursor at a time
constexpr uint32_t kMegaChunk = 64u;

// four waves per SIMD instead of the three the register count would give:
// a few spilled registers cost less than the lost latency hiding
template <int LDS, bool COUNT, int WAVES, bool INST, bool ATTR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES))) k_mega(SceneView sc, CamView cam, PathParams pp, float* __restrict__ img,
                                              float* __restrict__ acc, uint2* __restrict__ ovf, int gcap,
                                              uint32_t* __restrict__ stats, unsigned long long* __restrict__ trav,
                                              int xcd_local) {
    extern __shared__ __align__(8) uint32_t smem[];
    const uint32_t nlanes = gridDim.x * blockDim.x;
    const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
    TravStack<LDS, COUNT> st = make_stack<LDS, COUNT>(smem, ovf, gcap, gtid, nlanes);
    __shared__ uint32_t light_buf[3 * kLdsLights];
    const LightCache lc = stage_lights(sc, light_buf);
    const uint32_t npix = (uint32_t)cam.W * (uint32_t)cam.H;
    uint32_t n_ext = 0, n_sh = 0;
    // One loop trip = one path vertex.  A lane whose path ends starts its
    // next sample on the next trip instead of waiting for the longest path
    // of its wave; a lane whose pixel is done takes the next pixel of its
    // wave's chunk, and a wave whose chunk is used up takes the next
    // kMegaChunk pixels from a global cursor (one atomic per chunk), so
    // lanes and waves stay busy until the frame is drained.  A pixel's
    // samples still run in order on one lane, so its sum is the same.
    // With xcd_local the frame's pixels are split into eight bands of rows,
    // one cursor each (stats + 8 ...); the waves of XCD x (workgroups b with
    // b mod 8 = x) take chunks from band x first, so neighbouring pixels
    // share that XCD's L2, and then help with the other bands in turn.
    unsigned long long* cursor = reinterpret_cast<unsigned long long*>(stats + 4);
    const uint32_t nbands = xcd_local ? 8u : 1u;
    const uint32_t band_px = (npix + nbands - 1u) / nbands;
    uint32_t band = xcd_local ? (blockIdx.x & 7u) : 0u, bands_left = nbands;  // wave-uniform
    uint32_t next = 0, end = 0;  // this wave's chunk (wave-uniform)
    bool drained = false;        // every band's cursor has passed its last pixel (wave-uniform)
    bool live = false;
    uint32_t pix = 0, s = 0;
    f3 sum = mk3(0.f, 0.f, 0.f);
    PathRun pr;
    bool started = false;
    while (true) {
        const uint64_t idle = __ballot(!live);
        if (idle != 0ull && !drained) {
            while (next >= end && !drained) {
                const uint32_t lo = band * band_px, hi = min(lo + band_px, npix);
                unsigned long long base = 0ull;
                if (lane_id() == 0) base = atomicAdd(cursor + (xcd_local ? 2u + band : 0u), (unsigned long long)kMegaChunk);
                base = wave_broadcast_u64(base) + lo;
                if (base >= (unsigned long long)hi) {
                    // this band is done: the next one, until all are
                    if (--bands_left == 0u) drained = true;
                    band = band + 1u == nbands ? 0u : band + 1u;
                } else {
                    next = (uint32_t)base;
                    end = (uint32_t)min(base + (unsigned long long)kMegaChunk, (unsigned long long)hi);
                }
            }
            if (!drained) {
                if (!live) {
                    const uint32_t pos = next + rank_in(idle);
                    if (pos < end) {
                        pix = pos;
                        s = 0;
                        started = false;
                        live = true;
                    }
                }
                next = min(next + (uint32_t)__popcll(idle), end);
            }
        }
        if (__ballot(live) == 0ull) {
            if (drained) break;
            continue;
        }
        if (!live) continue;
        const uint32_t sample = pp.frame * (uint32_t)pp.spp + s;
        if (!started) {
            path_begin(cam, pp, pix, sample, pr);
            started = true;
        }
        if (path_vertex<LDS, COUNT, INST, ATTR>(sc, pp, pix, sample, pr, st, n_ext, n_sh, lc)) continue;
        started = false;
        sum = s == 0 ? pr.ps.L : add3(sum, pr.ps.L);
        if (++s == (uint32_t)pp.spp) {
            const float fs = (float)pp.spp;
            store_pixel(img, acc, pix, mk3(sum.x / fs, sum.y / fs, sum.z / fs), pp.frame);
            live = false;
        }
    }
    // ray counts: one atomic per wave for the whole kernel
    uint32_t e = n_ext, sh = n_sh;
    for (int off = 32; off > 0; off >>= 1) {
        e += __shfl_xor(e, off);
        sh += __shfl_xor(sh, off);
    }
    if ((gtid & 63u) == 0 && (e | sh)) {
        atomicAdd(&stats[0], e);
        atomicAdd(&stats[1], sh);
    }
    if constexpr (COUNT) {
        wave_add_u64(&trav[0], st.nodes);
        wave_add_u64(&trav[1], st.tris);
    }
    if (st.overflow) atomicOr(&stats[2], 1u);
}

// ---------------------------------------------------------------------------
// wavefront stages
// ---------------------------------------------------------------------------
__global__ void k_init_counts(uint32_t* __restrict__ counts, int n, uint32_t first) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) counts[i] = i == 0 ? first : 0u;
}

// The paper's two-slot count buffer (ablation): after a bounce, the next
// bounce's live count moves from slot + 1 to slot, slot + 1 is cleared, and
// the count is also kept at [b + 1] for the frame statistics.  b = -1 (the
// frame start): the slot takes [0], the initial paths.
__global__ void k_promote(WaveBufs wb, int b) {
    uint32_t* c = wb.counts;
    if (b < 0) {
        c[wb.slot] = c[0];
    } else {
        c[b + 1] = c[wb.slot + 1];
        c[wb.slot] = c[wb.slot + 1];
    }
    c[wb.slot + 1] = 0u;
}

// hybrid tail: a queue with fewer than `tail` paths is too short to keep
// the stage kernels busy; each path is shaded and finished in place.
// Limited to 128 VGPRs (4 waves per SIMD, a few spilled registers): at 148
// it ran 3 waves per SIMD and kept the next frame's stage kernels off the
// compute units while it finished the last bounces.
template <int LDS, bool COUNT, bool INST, bool ATTR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_shade_tail(SceneView sc, PathParams pp, WaveBufs wb, int b, int sorted,
                                                    uint32_t tail, uint2* __restrict__ ovf, int gcap,
                                                    uint32_t spread) {
    const uint32_t count = wb.counts[live_slot(wb, b)];
    if (!(count < tail) || count == 0u) return;
    extern __shared__ __align__(8) uint32_t smem[];
    __shared__ uint32_t light_buf[3 * kLdsLights];
    const LightCache lc = stage_lights(sc, light_buf);
    const uint32_t nlanes = gridDim.x * blockDim.x;
    const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t* perm = (sorted && wb.hist[2 * kSortBins]) ? wb.perm : nullptr;
    TravStack<LDS, COUNT> st = make_stack<LDS, COUNT>(smem, ovf, gcap, gtid, nlanes);
    uint32_t n_ext = 0, n_sh = 0;
    // spread = 0: entry i goes to thread i (full waves).  spread > 0: entry
    // i goes to lane i / spread of wave i % spread, so a short queue is
    // spread over the first `spread` waves (as many as the compute units
    // hold at once): every SIMD then has several waves whose memory latency
    // it can overlap, at the price of partly filled waves.  Either way one
    // lane finishes each path.
    const uint32_t wave = gtid >> 6;
    const uint32_t first = spread ? lane_id() * spread + wave : gtid;
    const uint32_t step = spread ? 64u * spread : nlanes;
    const bool takes = spread == 0u || wave < spread;
    for (uint32_t i = first; takes && i < count; i += step) {
        VertexOut vo;
        ShadowReq sh;
        PathState ps;
        const uint32_t path = shade_item<INST, ATTR>(sc, pp, wb, b, i, vo, sh, ps, perm, lc, true);
        finish_path<LDS, COUNT, INST, ATTR>(sc, pp, wb, path, b + 1, vo, sh, ps, st, n_ext, n_sh, lc);
    }
    // every lane of the wave is here: reduce the ray counts across it
    for (int off = 32; off > 0; off >>= 1) {
        n_ext += __shfl_xor(n_ext, off);
        n_sh += __shfl_xor(n_sh, off);
    }
    if (lane_id() == 0 && (n_ext | n_sh)) {
        atomicAdd(&wb.counts[wb.tail_slot], n_ext);
        atomicAdd(&wb.counts[wb.tail_slot + 1], n_sh);
    }
    if constexpr (COUNT) {
        wave_add_u64(&wb.trav[4], st.nodes);
        wave_add_u64(&wb.trav[5], st.tris);
    }
    if (st.overflow) atomicOr(&wb.counts[wb.err_slot], 1u);
}

__global__ void __launch_bounds__(256) k_raygen(CamView cam, PathParams pp, WaveBufs wb) {
    const uint32_t nlanes = gridDim.x * blockDim.x;
    const uint32_t npaths = (uint32_t)cam.W * (uint32_t)cam.H * (uint32_t)pp.spp;
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < npaths; p += nlanes) raygen_item(cam, pp, wb, p);
}

// Persistent traversal: each wave owns a contiguous chunk of the queue and
// keeps its 64 lanes busy by handing queue entries to lanes whose ray has
// finished, one traversal step per loop trip, instead of letting finished
// lanes idle until the slowest ray of the wave is done.  Lanes are refilled
// when at least `refill` of them are idle (or all are); the chunk cursor is
// wave-uniform, so no atomics are needed.

template <int LDS, bool COUNT, bool INST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) k_extend(SceneView sc, WaveBufs wb, int b, uint2* __restrict__ ovf, int gcap,
                                                uint32_t refill, int sorted, int xcd_local) {
    extern __shared__ __align__(8) uint32_t smem[];
    const uint32_t nlanes = gridDim.x * blockDim.x;
    const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
    TravStack<LDS, COUNT> st = make_stack<LDS, COUNT>(smem, ovf, gcap, gtid, nlanes);
    const int cur = b & 1;
    // with a ray sort this bounce, position i of the queue is slot perm[i]
    const uint32_t* perm = (sorted && wb.hist[2 * kSortBins]) ? wb.perm : nullptr;
    uint32_t next, end;
    wave_chunk(wb.counts[live_slot(wb, b)], next, end, xcd_local);
    bool live = false;
    uint32_t item = 0, ref = 0;
    Ray ray;
    Hit h;
    InstTrav it;
    while (true) {
        const uint64_t idle = __ballot(!live);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (next < end && (nidle >= refill || nidle == 64u)) {
            if (!live) {
                const uint32_t pos = next + rank_in(idle);
                if (pos < end) {
                    const uint32_t i = perm ? perm[pos] : pos;
                    // both loads issued before either is used (one wait)
                    const float4 o4 = wb.ray_o[cur][i];
                    const float4 d4 = wb.ray_d[cur][i];
                    if (f2u(o4.w) != kDeadPath) {  // dead slots (no compaction) need no hit
                        if constexpr (INST) {
                            closest_begin_inst<LDS>(xyz(o4), xyz(d4), INFINITY, ray, it, h, ref, st);
                        } else {
                            ray = make_ray(xyz(o4), xyz(d4));
                            closest_begin<LDS>(INFINITY, h, ref, st);
                        }
                        item = i;
                        live = true;
                    }
                }
            }
            next = min(next + nidle, end);
        }
        if (__ballot(live) == 0ull) {
            if (next < end) continue;
            break;
        }
        if constexpr (INST) {
            if (live && !closest_step_inst<LDS>(sc, ray, it, INFINITY, h, ref, st)) {
                wb.hit[item] = make_float4(h.t, u2f(h.inst), 0.f, u2f(h.tri));
                live = false;
            }
        } else {
            if (live && !closest_step<LDS>(sc, ray, INFINITY, h, ref, st)) {
                wb.hit[item] = make_float4(h.t, 0.f, 0.f, u2f(h.tri));
                live = false;
            }
        }
    }
    if constexpr (COUNT) {
        wave_add_u64(&wb.trav[0], st.nodes);
        wave_add_u64(&wb.trav[1], st.tris);
    }
    if (st.overflow) atomicOr(&wb.counts[wb.err_slot], 1u);
}

// Four waves per SIMD (at most 128 VGPRs, a few spilled): at the 137 it
// needs otherwise it ran three, and the stage took 17 % longer.
template <bool INST, bool ATTR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_shade(SceneView sc, PathParams pp, WaveBufs wb, int b, int compact,
                                               int sorted, uint32_t tail) {
    const uint32_t nlanes = gridDim.x * blockDim.x;
    const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t count = wb.counts[live_slot(wb, b)];
    if (compact && count < tail) return;  // k_shade_tail finishes this queue
    if (count == 0u) return;
    __shared__ uint32_t light_buf[3 * kLdsLights];
    const LightCache lc = stage_lights(sc, light_buf);
    const uint32_t* perm = (sorted && wb.hist[2 * kSortBins]) ? wb.perm : nullptr;
    const int nxt = (b & 1) ^ 1;
    uint32_t* next_count = &wb.counts[next_slot(wb, b)];
    uint32_t* sh_count = &wb.counts[wb.sh_base + b];
    if (!compact && gtid == 0 && count) atomicMax(next_count, count);
    // Queue slots are reserved once per block and trip, not once per wave:
    // concurrent atomics on one counter are serialised by the memory
    // system, and the shade stage issues two of them for every 64 paths
    // otherwise.  Block-uniform trip count (the block synchronises); the
    // per-wave counts are double-buffered by trip parity.
    __shared__ BlockReserve br;
    int par = 0;
    for (uint32_t bbase = blockIdx.x * blockDim.x; bbase < count; bbase += nlanes, par ^= 1) {
        const uint32_t i = bbase + threadIdx.x;
        VertexOut vo;
        ShadowReq sh;
        PathState ps;
        vo.cont = false;
        sh.valid = false;
        uint32_t path = kDeadPath;
        if (i < count) path = shade_item<INST, ATTR>(sc, pp, wb, b, i, vo, sh, ps, perm, lc);
        const uint64_t mk = compact ? __ballot(vo.cont) : 0ull;
        const uint64_t ms = __ballot(sh.valid);
        uint32_t jc, js;
        block_reserve2(br, par, next_count, mk, sh_count, ms, jc, js);
        if (compact) {
            if (vo.cont) write_continuation(wb, nxt, jc, vo, ps, path);
        } else if (i < count) {
            // no compaction: slots stay in place, finished paths marked dead
            if (vo.cont) write_continuation(wb, nxt, i, vo, ps, path);
            else write_dead(wb, nxt, i);
        }
        if (sh.valid) write_shadow(wb, js, sh, path);
    }
}

template <int LDS, bool COUNT, bool INST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) k_shadow(SceneView sc, WaveBufs wb, int b, uint2* __restrict__ ovf, int gcap,
                                                uint32_t refill, int xcd_local) {
    extern __shared__ __align__(8) uint32_t smem[];
    const uint32_t nlanes = gridDim.x * blockDim.x;
    const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
    TravStack<LDS, COUNT> st = make_stack<LDS, COUNT>(smem, ovf, gcap, gtid, nlanes);
    uint32_t next, end;
    wave_chunk(wb.counts[wb.sh_base + b], next, end, xcd_local);
    bool live = false;
    uint32_t item = 0, ref = 0;
    Ray ray;
    InstTrav it;
    while (true) {
        const uint64_t idle = __ballot(!live);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (next < end && (nidle >= refill || nidle == 64u)) {
            if (!live) {
                const uint32_t i = next + rank_in(idle);
                if (i < end) {
                    ray = make_ray(xyz(wb.sh_o[i]), xyz(wb.sh_d[i]));
                    if constexpr (INST) inst_begin(ray.o, ray.d, it);
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
        if (live) {
            bool occluded = false;
            bool more;
            if constexpr (INST) more = any_step_inst<LDS>(sc, ray, it, kShadowTmax, ref, st, occluded);
            else more = any_step<LDS>(sc, ray, kShadowTmax, ref, st, occluded);
            if (!more) {
                live = false;
                if (!occluded) shadow_add(wb, item);
                shadow_record(wb, b, item, !occluded);
            }
        }
    }
    if constexpr (COUNT) {
        wave_add_u64(&wb.trav[2], st.nodes);
        wave_add_u64(&wb.trav[3], st.tris);
    }
    if (st.overflow) atomicOr(&wb.counts[wb.err_slot], 1u);
}

// frame image I (written by the megakernel into a workspace slot) to the
// output image and the running average, in frame order
__global__ void __launch_bounds__(256) k_average(const float* __restrict__ I, uint32_t npix, uint32_t frame,
                                                 float* __restrict__ img, float* __restrict__ acc) {
    const uint32_t nlanes = gridDim.x * blockDim.x;
    for (uint32_t pix = blockIdx.x * blockDim.x + threadIdx.x; pix < npix; pix += nlanes)
        store_pixel(img, acc, pix, mk3(I[3 * (size_t)pix], I[3 * (size_t)pix + 1], I[3 * (size_t)pix + 2]), frame);
}

// ---------------------------------------------------------------------------
// material sort of a shade queue: histogram, scan, scatter of a permutation
// ---------------------------------------------------------------------------
// key 0: material of the hit (shade queue), 1: ray direction octant and
// origin side (extend queue)
__global__ void __launch_bounds__(256) k_sort_hist(SceneView sc, WaveBufs wb, int b, uint32_t threshold, int key_kind) {
    __shared__ uint32_t h[kSortBins];
    const uint32_t count = wb.counts[live_slot(wb, b)];
    if (count < threshold) return;
    for (int t = threadIdx.x; t < kSortBins; t += blockDim.x) h[t] = 0u;
    __syncthreads();
    const uint32_t nlanes = gridDim.x * blockDim.x;
    const int cur = b & 1;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += nlanes) {
        const uint32_t key = key_kind ? ray_key(sc, wb.ray_o[cur][i], wb.ray_d[cur][i]) : material_key(sc, wb.hit[i]);
        wb.sort_key[i] = key;
        atomicAdd(&h[key], 1u);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kSortBins; t += blockDim.x)
        if (h[t]) atomicAdd(&wb.hist[t], h[t]);
}

// one block of 64 threads: exclusive scan of the histogram into the running
// offsets, histogram cleared for the next bounce, sorted flag set
__global__ void k_sort_scan(WaveBufs wb, int b, uint32_t threshold) {
    __shared__ uint32_t v[kSortBins];
    const int t = threadIdx.x;
    const bool active = wb.counts[live_slot(wb, b)] >= threshold;
    v[t] = active ? wb.hist[t] : 0u;
    __syncthreads();
    for (int off = 1; off < kSortBins; off <<= 1) {
        uint32_t x = t >= off ? v[t - off] : 0u;
        __syncthreads();
        v[t] += x;
        __syncthreads();
    }
    wb.hist[kSortBins + t] = t == 0 ? 0u : v[t - 1];
    wb.hist[t] = 0u;
    if (t == 0) wb.hist[2 * kSortBins] = active ? 1u : 0u;
}

// per chunk of blockDim slots: block-local ranks in LDS, one global atomic
// per non-empty bin, then perm[offset + rank] = slot
__global__ void __launch_bounds__(256) k_sort_scatter(WaveBufs wb, int b, uint32_t threshold) {
    __shared__ uint32_t cnt[kSortBins], base[kSortBins];
    const uint32_t count = wb.counts[live_slot(wb, b)];
    if (count < threshold) return;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t c0 = blockIdx.x * blockDim.x; c0 < count; c0 += stride) {
        for (int t = threadIdx.x; t < kSortBins; t += blockDim.x) cnt[t] = 0u;
        __syncthreads();
        const uint32_t i = c0 + threadIdx.x;
        uint32_t key = 0, rank = 0;
        if (i < count) {
            key = wb.sort_key[i];
            rank = atomicAdd(&cnt[key], 1u);
        }
        __syncthreads();
        for (int t = threadIdx.x; t < kSortBins; t += blockDim.x)
            if (cnt[t]) base[t] = atomicAdd(&wb.hist[kSortBins + t], cnt[t]);
        __syncthreads();
        if (i < count) wb.perm[base[key] + rank] = i;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_accumulate(CamView cam, PathParams pp, const float4* __restrict__ L,
                                                    float* __restrict__ img, float* __restrict__ acc) {
    const uint32_t nlanes = gridDim.x * blockDim.x;
    const uint32_t npix = (uint32_t)cam.W * (uint32_t)cam.H;
    for (uint32_t pix = blockIdx.x * blockDim.x + threadIdx.x; pix < npix; pix += nlanes)
        accumulate_item(pp, L, img, acc, pix);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define PT_STACK_CASES(X) X(8) X(16) X(24) X(32)
// instantiate a traversal kernel for the LDS stack depth, the work-counting
// flag and the scene kind (flat / two-level)
#define PT_DISPATCH(N, launch) \
    if (lds == N) {            \
        if (sc.n_inst > 0) {   \
            if (count) launch(N, true, true) else launch(N, false, true)   \
        } else {               \
            if (count) launch(N, true, false) else launch(N, false, false) \
        }                      \
        return hipGetLastError(); \
    }

// the same for kernels that shade, which also take the attribute flag
#define PT_DISPATCH_SHADE(N, launch)                                                \
    if (lds == N) {                                                                 \
        const bool inst = sc.n_inst > 0, attr = sc.attr_flags != 0;                 \
        if (inst && attr) {                                                         \
            if (count) launch(N, true, true, true) else launch(N, false, true, true)   \
        } else if (inst) {                                                          \
            if (count) launch(N, true, true, false) else launch(N, false, true, false) \
        } else if (attr) {                                                          \
            if (count) launch(N, true, false, true) else launch(N, false, false, true) \
        } else {                                                                    \
            if (count) launch(N, true, false, false) else launch(N, false, false, false) \
        }                                                                           \
        return hipGetLastError();                                                   \
    }

static size_t stack_lds_bytes(int lds, int block) { return trav_stack_lds_bytes(lds, block); }

hipError_t launch_mega(int lds, bool count, int waves, dim3 grid, dim3 block, hipStream_t s, const SceneView& sc,
                       const CamView& cam, const PathParams& pp, float* img, float* acc, uint2* ovf, int gcap,
                       uint32_t* stats, unsigned long long* trav, int xcd_local) {
    size_t sm = stack_lds_bytes(lds, block.x);
#define L(N, C, I, A)                                                                                                \
    if (waves == 5)                                                                                                  \
        hipLaunchKernelGGL((k_mega<N, C, 5, I, A>), grid, block, sm, s, sc, cam, pp, img, acc, ovf, gcap, stats,     \
                           trav, xcd_local);                                                                         \
    else                                                                                                             \
        hipLaunchKernelGGL((k_mega<N, C, 4, I, A>), grid, block, sm, s, sc, cam, pp, img, acc, ovf, gcap, stats,     \
                           trav, xcd_local);
#define X(N) PT_DISPATCH_SHADE(N, L)
    PT_STACK_CASES(X)
#undef X
#undef L
    return hipErrorInvalidValue;
}

hipError_t launch_promote(hipStream_t s, const WaveBufs& wb, int b) {
    hipLaunchKernelGGL(k_promote, dim3(1), dim3(1), 0, s, wb, b);
    return hipGetLastError();
}

hipError_t launch_init_counts(hipStream_t s, uint32_t* counts, int n, uint32_t first) {
    hipLaunchKernelGGL(k_init_counts, dim3((n + 255) / 256), dim3(256), 0, s, counts, n, first);
    return hipGetLastError();
}

hipError_t launch_raygen(dim3 grid, dim3 block, hipStream_t s, const CamView& cam, const PathParams& pp,
                         const WaveBufs& wb) {
    hipLaunchKernelGGL(k_raygen, grid, block, 0, s, cam, pp, wb);
    return hipGetLastError();
}

hipError_t launch_extend(int lds, bool count, dim3 grid, dim3 block, hipStream_t s, const SceneView& sc,
                         const WaveBufs& wb, int b, uint2* ovf, int gcap, int sorted, int xcd_local) {
    size_t sm = stack_lds_bytes(lds, block.x);
#define L(N, C, I) hipLaunchKernelGGL((k_extend<N, C, I>), grid, block, sm, s, sc, wb, b, ovf, gcap, kRefill, sorted, xcd_local);
#define X(N) PT_DISPATCH(N, L)
    PT_STACK_CASES(X)
#undef X
#undef L
    return hipErrorInvalidValue;
}

hipError_t launch_shade(dim3 grid, dim3 block, hipStream_t s, const SceneView& sc, const PathParams& pp,
                        const WaveBufs& wb, int b, int compact, int sorted, uint32_t tail) {
    const uint32_t t = compact ? tail : 0u;
    if (sc.n_inst > 0 && sc.attr_flags)
        hipLaunchKernelGGL((k_shade<true, true>), grid, block, 0, s, sc, pp, wb, b, compact, sorted, t);
    else if (sc.n_inst > 0)
        hipLaunchKernelGGL((k_shade<true, false>), grid, block, 0, s, sc, pp, wb, b, compact, sorted, t);
    else if (sc.attr_flags)
        hipLaunchKernelGGL((k_shade<false, true>), grid, block, 0, s, sc, pp, wb, b, compact, sorted, t);
    else
        hipLaunchKernelGGL((k_shade<false, false>), grid, block, 0, s, sc, pp, wb, b, compact, sorted, t);
    return hipGetLastError();
}

hipError_t launch_tail(int lds, bool count, dim3 grid, dim3 block, hipStream_t s, const SceneView& sc,
                       const PathParams& pp, const WaveBufs& wb, int b, int sorted, uint32_t tail, uint2* ovf,
                       int gcap, uint32_t resident_waves) {
    const size_t sm = stack_lds_bytes(lds, block.x);
    const uint32_t spread = resident_waves ? std::max(1u, std::min(grid.x * block.x / 64u, resident_waves)) : 0u;
#define L(N, C, I, A) hipLaunchKernelGGL((k_shade_tail<N, C, I, A>), grid, block, sm, s, sc, pp, wb, b, sorted, tail, ovf, gcap, spread);
#define X(N) PT_DISPATCH_SHADE(N, L)
    PT_STACK_CASES(X)
#undef X
#undef L
    return hipErrorInvalidValue;
}

hipError_t launch_sort(dim3 grid, dim3 block, hipStream_t s, const SceneView& sc, const WaveBufs& wb, int b,
                       uint32_t threshold, int key_kind) {
    hipLaunchKernelGGL(k_sort_hist, grid, block, 0, s, sc, wb, b, threshold, key_kind);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(kSortBins), 0, s, wb, b, threshold);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_scatter, grid, block, 0, s, wb, b, threshold);
    return hipGetLastError();
}

hipError_t launch_shadow(int lds, bool count, dim3 grid, dim3 block, hipStream_t s, const SceneView& sc,
                         const WaveBufs& wb, int b, uint2* ovf, int gcap, int xcd_local) {
    size_t sm = stack_lds_bytes(lds, block.x);
#define L(N, C, I) hipLaunchKernelGGL((k_shadow<N, C, I>), grid, block, sm, s, sc, wb, b, ovf, gcap, kRefill, xcd_local);
#define X(N) PT_DISPATCH(N, L)
    PT_STACK_CASES(X)
#undef X
#undef L
    return hipErrorInvalidValue;
}

hipError_t launch_average(dim3 grid, dim3 block, hipStream_t s, const float* I, uint32_t npix, uint32_t frame,
                          float* img, float* acc) {
    hipLaunchKernelGGL(k_average, grid, block, 0, s, I, npix, frame, img, acc);
    return hipGetLastError();
}

hipError_t launch_accumulate(dim3 grid, dim3 block, hipStream_t s, const CamView& cam, const PathParams& pp,
                             const float4* L, float* img, float* acc) {
    hipLaunchKernelGGL(k_accumulate, grid, block, 0, s, cam, pp, L, img, acc);
    return hipGetLastError();
}

}  // namespace ptmi
