// Adjoint kernels of libptmi: replay A of every camera path sample (its
// radiance, kept per path), then replay B from the same random numbers,
// gradients added with hardware fp32 atomics (see adjoint.h for the
// algorithm).
#include "adjoint.h"
#include "wave.h"
#include "kernels.h"

namespace ptmi {

namespace {

// Gradients go to global memory with hardware fp32 atomics, except two
// kinds of hot spots, which each block sums in LDS and adds once at the
// end: the light-sample emission terms of lights in the first kLdsLights
// entries of the light table (every visible light sample adds to one of
// them), and the albedo and emission terms of the kHotTris largest
// triangles (a ground plane or an area light is reached by a large share
// of all paths, and atomics on a few addresses are served one at a time).
struct AtomicAcc {
    float* lds_light;  // 3 floats per light (local memory of the block)
    uint32_t n_lds;    // lights kept there
    float* lds_hot;    // [albedo, emission][3 * kHotTris] sums of the largest triangles
    uint32_t n_hot;
    __device__ __forceinline__ void add_tri(uint32_t hot, int which, int c, float* p, float v) {
        if (v == 0.0f) return;
        if (hot - 1u < n_hot)
            atomicAdd(&lds_hot[which * 3 * kHotTris + 3 * (hot - 1u) + (uint32_t)c], v);
        else
            unsafeAtomicAdd(p, v);
    }
    __device__ __forceinline__ void add_light(uint32_t j, int c, float* p, float v) {
        if (v == 0.0f) return;
        if (j < n_lds)
            atomicAdd(&lds_light[3 * j + (uint32_t)c], v);
        else
            unsafeAtomicAdd(p, v);
    }
};

}  // namespace

// Replay A of every path: its radiance, into Lpath[path].  One loop trip =
// one path vertex; a lane whose path is done takes the next path of its
// wave's chunk, a wave whose chunk is used up takes the next 64 paths from
// cursor[0].  Five waves per SIMD, as the megakernel.  STORE: every
// vertex's intersection and light-sample visibility go to rec as well.
template <int LDS, bool ATTR, bool STORE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) k_adjoint_radiance(
    SceneView sc, CamView cam, PathParams pp, float4* __restrict__ Lpath, unsigned long long* __restrict__ cursor,
    uint2* __restrict__ ovf, int gcap, uint32_t* __restrict__ stats, VertexRecs rec) {
    extern __shared__ __align__(8) uint32_t smem[];
    const uint32_t nlanes = gridDim.x * blockDim.x;
    const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
    TravStack<LDS> st =
        make_trav_stack<LDS>(reinterpret_cast<uint2*>(smem) + threadIdx.x, (int)blockDim.x, ovf, gtid, (int)nlanes, gcap);
    const uint32_t npaths = (uint32_t)cam.W * (uint32_t)cam.H * (uint32_t)pp.spp;
    uint32_t next = 0, end = 0;  // wave-uniform
    bool drained = false;        // wave-uniform
    bool live = false;
    uint32_t path = 0, pix = 0, sample = 0, ne = 0, ns = 0;
    PathRun pr;
    while (true) {
        const uint64_t idle = __ballot(!live);
        if (idle != 0ull && !drained) {
            if (next >= end) {
                unsigned long long base = 0ull;
                if (lane_id() == 0) base = atomicAdd(cursor, 64ull);
                base = wave_broadcast_u64(base);
                if (base >= (unsigned long long)npaths) {
                    drained = true;
                } else {
                    next = (uint32_t)base;
                    end = (uint32_t)min(base + 64ull, (unsigned long long)npaths);
                }
            }
            if (!drained) {
                if (!live) {
                    const uint32_t p = next + rank_in(idle);
                    if (p < end) {
                        path = p;
                        pix = p / (uint32_t)pp.spp;
                        sample = pp.frame * (uint32_t)pp.spp + (p - pix * (uint32_t)pp.spp);
                        path_begin(cam, pp, pix, sample, pr);
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
        if constexpr (STORE) {
            if (adjoint_a_vertex<LDS, ATTR>(sc, pp, pix, sample, path, pr, st, ne, ns, rec)) continue;
        } else {
            if (path_vertex<LDS, false, false, ATTR>(sc, pp, pix, sample, pr, st, ne, ns)) continue;
        }
        Lpath[path] = make_float4(pr.ps.L.x, pr.ps.L.y, pr.ps.L.z, 0.f);
        live = false;
    }
    // the rays of the paths (replay B traces the same ones again): one
    // atomic per wave for the whole kernel
    for (int off = 32; off > 0; off >>= 1) {
        ne += __shfl_xor(ne, off);
        ns += __shfl_xor(ns, off);
    }
    if (lane_id() == 0 && (ne | ns)) {
        atomicAdd(&stats[0], ne);
        atomicAdd(&stats[1], ns);
    }
    if (st.overflow) atomicOr(&stats[2], 1u);
}

// Replay B of every path, one vertex per loop trip with the same hand-out
// of paths (cursor[1]), from the radiance replay A left in Lpath.  STORED:
// from replay A's records too, tracing no ray (no traversal stack, so its
// register budget is set on its own).
constexpr int kStoredWaves = 4;

template <int LDS, bool ATTR, bool STORED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(STORED ? kStoredWaves : 4))) k_adjoint(SceneView sc, CamView cam, PathParams pp,
                                                 const float* __restrict__ d_img, const float4* __restrict__ Lpath,
                                                 unsigned long long* __restrict__ cursor, float* __restrict__ g_alb,
                                                 float* __restrict__ g_emi, uint2* __restrict__ ovf, int gcap,
                                                 uint32_t* __restrict__ stats, int count_rays, VertexRecs rec) {
    extern __shared__ __align__(8) uint32_t smem[];
    const uint32_t nlanes = gridDim.x * blockDim.x;
    const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
    TravStack<LDS> st =
        make_trav_stack<LDS>(reinterpret_cast<uint2*>(smem) + threadIdx.x, (int)blockDim.x, ovf, gtid, (int)nlanes, gcap);
    __shared__ float light_g[3 * kLdsLights];
    __shared__ float hot_g[2 * 3 * kHotTris];
    AtomicAcc acc;
    acc.lds_light = light_g;
    acc.n_lds = (uint32_t)min(max(sc.nl, 0), kLdsLights);
    acc.lds_hot = hot_g;
    acc.n_hot = (uint32_t)min(max(sc.n_hot, 0), kHotTris);
    for (uint32_t j = threadIdx.x; j < 3 * acc.n_lds; j += blockDim.x) light_g[j] = 0.0f;
    for (uint32_t j = threadIdx.x; j < 2 * 3 * kHotTris; j += blockDim.x) hot_g[j] = 0.0f;
    __syncthreads();
    const uint32_t npaths = (uint32_t)cam.W * (uint32_t)cam.H * (uint32_t)pp.spp;
    const float fs = (float)pp.spp;
    uint32_t next = 0, end = 0;  // wave-uniform
    bool drained = false;        // wave-uniform
    bool live = false;
    AdjRun ar;
    uint32_t ne = 0, ns = 0;
    while (true) {
        const uint64_t idle = __ballot(!live);
        if (idle != 0ull && !drained) {
            if (next >= end) {
                unsigned long long base = 0ull;
                if (lane_id() == 0) base = atomicAdd(cursor + 1, 64ull);
                base = wave_broadcast_u64(base);
                if (base >= (unsigned long long)npaths) {
                    drained = true;
                } else {
                    next = (uint32_t)base;
                    end = (uint32_t)min(base + 64ull, (unsigned long long)npaths);
                }
            }
            if (!drained) {
                if (!live) {
                    const uint32_t p = next + rank_in(idle);
                    if (p < end) {
                        const uint32_t pix = p / (uint32_t)pp.spp;
                        const uint32_t s = p - pix * (uint32_t)pp.spp;
                        const f3 delta = mk3(d_img[3 * (size_t)pix] / fs, d_img[3 * (size_t)pix + 1] / fs,
                                             d_img[3 * (size_t)pix + 2] / fs);
                        adjoint_b_begin(cam, pp, pix, pp.frame * (uint32_t)pp.spp + s, delta, xyz(Lpath[p]), ar, p);
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
        if (!adjoint_b_step<LDS, ATTR, AtomicAcc, false, STORED>(sc, pp, ar, g_alb, g_emi, st, acc, ne, ns, rec))
            live = false;
    }
    // with count_rays (replay A ran as the wavefront, which keeps its own
    // counters) the paths' rays are counted here (traced here, or by
    // replay A with its records), one atomic per wave
    if (count_rays) {
        for (int off = 32; off > 0; off >>= 1) {
            ne += __shfl_xor(ne, off);
            ns += __shfl_xor(ns, off);
        }
        if (lane_id() == 0 && (ne | ns)) {
            atomicAdd(&stats[0], ne);
            atomicAdd(&stats[1], ns);
        }
    }
    // every thread of the block is here: add the block's sums
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < 3 * acc.n_lds; j += blockDim.x) {
        const float v = light_g[j];
        if (v != 0.0f) unsafeAtomicAdd(g_emi + 3 * (size_t)sc.lights[j / 3u].id + j % 3u, v);
    }
    for (uint32_t j = threadIdx.x; j < 3 * acc.n_hot; j += blockDim.x) {
        const size_t at = 3 * (size_t)sc.hot_ids[j / 3u] + j % 3u;
        const float va = hot_g[j], ve = hot_g[3 * kHotTris + j];
        if (va != 0.0f) unsafeAtomicAdd(g_alb + at, va);
        if (ve != 0.0f) unsafeAtomicAdd(g_emi + at, ve);
    }
    if (st.overflow) atomicOr(&stats[2], 1u);
}

hipError_t launch_adjoint_radiance(int lds, dim3 grid, dim3 block, hipStream_t s, const SceneView& sc,
                                   const CamView& cam, const PathParams& pp, float4* Lpath,
                                   unsigned long long* cursor, uint2* ovf, int gcap, uint32_t* stats,
                                   const VertexRecs& rec) {
    size_t sm = trav_stack_lds_bytes(lds, (int)block.x);
#define K(N, A, S) \
    hipLaunchKernelGGL((k_adjoint_radiance<N, A, S>), grid, block, sm, s, sc, cam, pp, Lpath, cursor, ovf, gcap, stats, rec)
#define X(N)                                                  \
    if (lds == N) {                                           \
        if (rec.hit) {                                        \
            if (sc.attr_flags) K(N, true, true);              \
            else K(N, false, true);                           \
        } else {                                              \
            if (sc.attr_flags) K(N, true, false);             \
            else K(N, false, false);                          \
        }                                                     \
        return hipGetLastError();                             \
    }
    X(8) X(16) X(24) X(32)
#undef X
#undef K
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint(int lds, dim3 grid, dim3 block, hipStream_t s, const SceneView& sc, const CamView& cam,
                          const PathParams& pp, const float* d_img, const float4* Lpath, unsigned long long* cursor,
                          float* g_alb, float* g_emi, uint2* ovf, int gcap, uint32_t* stats, int count_rays,
                          const VertexRecs& rec) {
    // with the records replay B traces nothing: no traversal stack in LDS
    const size_t sm = rec.hit ? 0 : trav_stack_lds_bytes(lds, (int)block.x);
#define K(N, A, S)                                                                                               \
    hipLaunchKernelGGL((k_adjoint<N, A, S>), grid, block, sm, s, sc, cam, pp, d_img, Lpath, cursor, g_alb, g_emi, \
                       ovf, gcap, stats, count_rays, rec)
    if (rec.hit) {
        if (sc.attr_flags) K(8, true, true);
        else K(8, false, true);
        return hipGetLastError();
    }
#define X(N)                                      \
    if (lds == N) {                               \
        if (sc.attr_flags) K(N, true, false);     \
        else K(N, false, false);                  \
        return hipGetLastError();                 \
    }
    X(8) X(16) X(24) X(32)
#undef X
#undef K
    return hipErrorInvalidValue;
}

}  // namespace ptmi
