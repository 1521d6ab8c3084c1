// Kernel launchers of libptmi (definitions in kernels.hip).
#pragma once
#include "../../include/ptmi.h"
#include "device.h"
#include "adjoint.h"

namespace ptmi {

constexpr uint32_t kDeadPath = 0xFFFFFFFFu;

// Wavefront path state, structure of arrays (one float4 stream per field
// group, so that a wave's 64 lanes read or write 1 KiB contiguously).
//   ray_o[q][i] = (origin, path id)     ray_d[q][i] = (direction, last pdf)
//   pst[q][i]   = (throughput, flags)   hit[i] = (t, 0, 0, leaf-order tri)
//   (the shade stage recomputes the hit's barycentrics, hit_barycentrics)
//   sh_o/sh_d/sh_c[i] = shadow segment origin + path id, direction, beta*C
//   L[path]     = radiance of the path (indexed by path id, not queue slot)
// q alternates between bounces (ping-pong queues).
struct WaveBufs {
    float4* ray_o[2];
    float4* ray_d[2];
    float4* pst[2];
    float4* hit;
    float4* sh_o;
    float4* sh_d;
    float4* sh_c;
    float4* L;
    // [b] live paths at bounce b, [sh_base + b] shadow rays, [tail_slot] and
    // [tail_slot + 1] extension and shadow rays traced by the hybrid tail,
    // [err_slot] traversal stack overflow flag
    uint32_t* counts;
    // two_slot != 0 (the paper's two-slot count buffer, an ablation): the
    // stage kernels read the live count from [slot] and add the next
    // bounce's to [slot + 1]; k_promote moves it over between bounces
    int two_slot, slot;
    // traversal work counters: node visits and triangle tests of the
    // extend [0, 1], shadow [2, 3] and hybrid-tail [4, 5] kernels
    unsigned long long* trav;
    int sh_base;
    int tail_slot;
    int err_slot;
    // material sort (optional): keys and permutation per queue slot, 64-bin
    // histogram / running offsets, flag = 1 when the current queue is sorted
    uint32_t* sort_key;
    uint32_t* perm;
    uint32_t* hist;     // [64] counts, [64..127] running offsets, [128] sorted flag
    // the adjoint's replay A with kept intersections (else null): vertex
    // k of path p at [(k - 1) * rec_n + p], its hit written by the shade
    // stage and the hybrid tail, its light-sample visibility by the shadow
    // stage and the tail (see VertexRecs)
    uint2* rec_hit;
    uint8_t* rec_vis;
    uint32_t rec_n;
};

constexpr int kSortBins = 64;

// the live count of bounce b and the next bounce's count
__host__ __device__ inline uint32_t live_slot(const WaveBufs& wb, int b) {
    return wb.two_slot ? (uint32_t)wb.slot : (uint32_t)b;
}
__host__ __device__ inline uint32_t next_slot(const WaveBufs& wb, int b) {
    return wb.two_slot ? (uint32_t)wb.slot + 1u : (uint32_t)b + 1u;
}
// persistent traversal kernels refill a wave's idle lanes once this many
// of its 64 lanes are idle
constexpr uint32_t kRefill = 16;

// stats: [0] extension rays, [1] shadow rays, [2] overflow flag; trav:
// node visits, triangle tests
// count: traversal kernels also count node visits and triangle tests
// waves: the megakernel's occupancy, 4 or 5 waves per SIMD
hipError_t launch_mega(int lds, bool count, int waves, dim3 grid, dim3 block, hipStream_t s, const SceneView& sc,
                       const CamView& cam, const PathParams& pp, float* img, float* acc, uint2* ovf, int gcap,
                       uint32_t* stats, unsigned long long* trav, int xcd_local);
hipError_t launch_promote(hipStream_t s, const WaveBufs& wb, int b);
hipError_t launch_init_counts(hipStream_t s, uint32_t* counts, int n, uint32_t first);
hipError_t launch_raygen(dim3 grid, dim3 block, hipStream_t s, const CamView& cam, const PathParams& pp,
                         const WaveBufs& wb);
// sorted: a ray sort of queue b precedes (its permutation orders the work)
hipError_t launch_extend(int lds, bool count, dim3 grid, dim3 block, hipStream_t s, const SceneView& sc,
                         const WaveBufs& wb, int b, uint2* ovf, int gcap, int sorted, int xcd_local);
// tail > 0 (compacted queues only): a queue with fewer than `tail` paths is
// skipped here and finished in place by launch_tail
hipError_t launch_shade(dim3 grid, dim3 block, hipStream_t s, const SceneView& sc, const PathParams& pp,
                        const WaveBufs& wb, int b, int compact, int sorted, uint32_t tail);
// resident_waves: 0 = queue entries in full waves; else the waves the
// device holds at once at the tail kernel's occupancy, over which a short
// queue is spread
hipError_t launch_tail(int lds, bool count, dim3 grid, dim3 block, hipStream_t s, const SceneView& sc,
                       const PathParams& pp, const WaveBufs& wb, int b, int sorted, uint32_t tail, uint2* ovf,
                       int gcap, uint32_t resident_waves);
// counting sort of queue b by a 6-bit key when it holds >= threshold
// paths: key_kind 0 = material of the hit (for shade), 1 = ray direction
// octant and origin side (for extend)
hipError_t launch_sort(dim3 grid, dim3 block, hipStream_t s, const SceneView& sc, const WaveBufs& wb, int b,
                       uint32_t threshold, int key_kind);
hipError_t launch_shadow(int lds, bool count, dim3 grid, dim3 block, hipStream_t s, const SceneView& sc,
                         const WaveBufs& wb, int b, uint2* ovf, int gcap, int xcd_local);
// the adjoint: replay A of every path into Lpath (one float4 per path;
// cursor[0], zero on entry), then replay B (cursor[1], zero on entry);
// with rec.hit set replay A keeps every vertex's intersection and
// light-sample visibility there and replay B reads them (no tracing)
hipError_t launch_adjoint_radiance(int lds, dim3 grid, dim3 block, hipStream_t s, const SceneView& sc,
                                   const CamView& cam, const PathParams& pp, float4* Lpath,
                                   unsigned long long* cursor, uint2* ovf, int gcap, uint32_t* stats,
                                   const VertexRecs& rec);
hipError_t launch_adjoint(int lds, dim3 grid, dim3 block, hipStream_t s, const SceneView& sc, const CamView& cam,
                          const PathParams& pp, const float* d_img, const float4* Lpath, unsigned long long* cursor,
                          float* g_alb, float* g_emi, uint2* ovf, int gcap, uint32_t* stats, int count_rays,
                          const VertexRecs& rec);
hipError_t launch_accumulate(dim3 grid, dim3 block, hipStream_t s, const CamView& cam, const PathParams& pp,
                             const float4* L, float* img, float* acc);
// img = I, running average acc updated for frame `frame` (npix pixels)
hipError_t launch_average(dim3 grid, dim3 block, hipStream_t s, const float* I, uint32_t npix, uint32_t frame,
                          float* img, float* acc);

struct BatchBufs;
hipError_t launch_batch_init(hipStream_t s, const BatchBufs& bb, uint32_t total);
hipError_t launch_batch_iteration(int lds, dim3 grid, dim3 block, hipStream_t s, const BatchBufs& bb, int q,
                                  uint2* ovf, int gcap, bool attr);
hipError_t launch_batch_accumulate(dim3 grid, dim3 block, hipStream_t s, const BatchBufs& bb, uint32_t total_pix);

}  // namespace ptmi
