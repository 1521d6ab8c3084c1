/*
 * ptmi: megakernel and wavefront Monte Carlo path tracing of triangle
 * scenes on AMD Instinct MI355X (gfx950), as a C-ABI shared library.
 *
 * What is computed (paper Sec. 2.1-2.3, Eq. 1-3): for every pixel p of a
 * W x H pinhole camera, the estimator
 *     I(p) = (1/spp) * sum_{s<spp} L(p, s)
 * of the light transport equation, where L(p, s) is one camera path traced
 * vertex by vertex (extend to the closest hit, add emitted radiance times
 * the throughput, sample a new direction and update the throughput, up to
 * max_depth scattering vertices).  Next-event estimation with the power
 * heuristic and Russian roulette are options.  Random numbers come from
 * Philox4x64-10 keyed by (pixel, frame * spp + s, bounce, job) under key
 * (seed, 0), so a path can be replayed exactly (the adjoint relies on it).
 *
 * Two schedules compute bit-identical images (paper Sec. 2.2-2.3, 3.1):
 *   PT_MODE_MEGA  one kernel; each thread traces its pixel's paths to the end.
 *   PT_MODE_WAVE  per bounce, separate extend / shade / shadow kernels over
 *                 structure-of-arrays path state in device memory, with the
 *                 live paths compacted into a queue after every bounce.
 *
 * Conventions
 *   - Every call returns a pt_status; 0 is success.  pt_last_error() gives
 *     a message for the calling thread.  No C++ exception crosses the ABI.
 *   - Host arrays passed in are copied; the caller keeps ownership.
 *   - All device memory is owned by the caller and passed as plain device
 *     pointers (for example from torch tensors); the library never
 *     allocates device memory.  Work is enqueued on the caller's HIP stream
 *     (a hipStream_t passed as void*; NULL = the null stream) and is
 *     asynchronous unless stated otherwise.
 *   - Asynchronous device errors surface at the next call or at pt_sync.
 *   - A context may be used by one host thread at a time.
 */
#ifndef PTMI_H
#define PTMI_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pt_status;
enum {
    PT_OK = 0,
    PT_EINVAL = -1,      /* bad argument */
    PT_ENOMEM = -2,      /* buffer or workspace too small */
    PT_EHIP = -3,        /* HIP runtime error or no GPU */
    PT_ESTATE = -4,      /* wrong call order (e.g. render before bind) */
    PT_EOVERFLOW = -5,   /* a device-side capacity was exceeded */
    PT_EUNSUPPORTED = -6 /* option not supported */
};

/* Material types.  PT_COATED (paper Sec. 3: a two-lobe subset of a layered
 * material such as OpenPBR's coat over a base): a GGX dielectric coat of the
 * material's roughness and ior over a Lambertian base of the triangle's
 * albedo, f = F(wo.h) D G2 / (4 cos_o cos_i) + (1 - F(cos_o)) (1 - F(cos_i))
 * albedo / pi with F the exact unpolarised Fresnel reflectance; sampled by
 * the coat's visible normals with probability F(cos_o), else the base's
 * cosine lobe. */
enum { PT_LAMBERT = 0, PT_CONDUCTOR = 1, PT_DIELECTRIC = 2, PT_COATED = 3 };
enum { PT_MODE_MEGA = 0, PT_MODE_WAVE = 1 };

/* Camera samplers (pt_render_args.sampler). */
enum { PT_SAMPLER_PHILOX = 0, PT_SAMPLER_HALTON = 1 };

/* Render flags (pt_render_args.flags). */
enum {
    PT_FLAG_PROFILE = 1,       /* time every stage launch with HIP events */
    PT_FLAG_NO_COMPACT = 2,    /* wavefront: no compaction, dispatch every path each bounce */
    PT_FLAG_SORT_MATERIAL = 4, /* wavefront: counting-sort each shade queue by material type */
    PT_FLAG_COUNT_WORK = 8,    /* traversal kernels count BVH node visits and triangle tests
                                  (pt_frame_stats); a separate kernel build, slower */
    PT_FLAG_SORT_RAYS = 16,    /* wavefront: counting-sort each extend queue by ray direction octant and
                                  origin side of the scene centre (coherent waves) */
    PT_FLAG_XCD_LOCAL = 32,    /* each of the eight XCDs (own L2 each) takes one contiguous part of the
                                  extend / shadow queues, and the megakernel's waves on an XCD take their
                                  pixels from one band of rows first; same image bit for bit */
    PT_FLAG_TWO_SLOT = 64,     /* wavefront, ablation of paper Sec. 3.1: the live path count in a
                                  two-slot buffer (current, next) that a one-thread promote kernel
                                  moves over after every bounce, in place of one counter per bounce;
                                  same image bit for bit */
    PT_FLAG_KEEP_HITS = 128,   /* backward: the first replay keeps every path vertex's intersection
                                  and light-sample visibility (9 bytes per vertex and path sample in
                                  the workspace) and the second reads them instead of tracing the
                                  same rays again; same gradients; ignored by forward renders */
    PT_FLAG_SERIAL_STAGES = 256 /* wavefront frame or backward: every stage on `stream`, the shadow
                                  stage not beside the next extend stage, so that each kernel's
                                  event time is its own (per-kernel measurement); same results */
};

typedef struct pt_ctx pt_ctx;

/* Triangle scene (paper Sec. 3: scene data packed on the CPU).
 * positions  float[nv*3]; indices int32[nt*3], counter-clockwise (v0,v1,v2)
 * faces the front; tri_material int32[nt] indexes materials float[nm*4]
 * = (type, roughness, ior, checker frequency): the frequency (>= 0; 0 =
 * none) textures the albedo of Lambertian and coated materials through the
 * vertex texture coordinates of pt_set_attributes; albedo and emission float[nt*3] per
 * triangle (emission is one-sided, front face only); sky float[3] is the
 * radiance of escaped rays.  Triangles with some emission channel > 0 at
 * load time form the fixed light set of next-event estimation (picked in
 * proportion to area).  Non-finite values or out-of-range indices give
 * PT_EINVAL. */
typedef struct {
    int32_t nv, nt, nm;
    const float* positions;
    const int32_t* indices;
    const int32_t* tri_material;
    const float* materials;
    const float* albedo;
    const float* emission;
    float sky[3];
} pt_scene_desc;

/* Two-level scene (paper Sec. 2.3 and 3: a top-level acceleration structure
 * over instances of per-mesh bottom-level structures).  Mesh m is the range
 * [mesh_first[m], mesh_first[m] + mesh_count[m]) of the loaded triangles
 * (object space; ranges may not overlap); instance q places mesh
 * inst_mesh[q] in the world by the affine map o2w[12 q .. 12 q + 11] (3x4
 * row-major: row r = three linear coefficients, then the translation) and
 * w2o (same layout) maps world rays into its object space.  The world is
 * then the instances: a ray is tested against an instance's mesh with the
 * object-space ray ((M0 x + M1 y) + M2 z) + M3 per row (direction without
 * translation, not renormalised, so t is the world ray's parameter); the
 * closest hit is the smallest t, ties to the smaller instance, then the
 * smaller triangle; shading, light sampling and light areas use the world
 * vertices o2w(v) in the same arithmetic; material, albedo and emission are
 * per mesh triangle and shared by the instances; the light set is every
 * (instance, emissive triangle) pair.  Call after pt_load_scene and before
 * pt_build_bvh; n_instances = 0 (or a NULL desc) returns to a flat scene.
 * The adjoint and the batched launch take flat scenes only
 * (PT_EUNSUPPORTED).  PT_EINVAL on out-of-range or overlapping ranges,
 * indices or non-finite matrices. */
typedef struct {
    int32_t n_meshes;
    const int32_t* mesh_first;
    const int32_t* mesh_count;
    int32_t n_instances;
    const int32_t* inst_mesh;
    const float* o2w;
    const float* w2o;
} pt_instances_desc;
pt_status pt_set_instances(pt_ctx* ctx, const pt_instances_desc* instances);

/* Vertex attributes (paper Sec. 2.3: the shading stage interpolates the
 * hit triangle's vertex normals and texture coordinates).  nv must equal
 * the loaded scene's vertex count; normals float[nv*3] and uvs float[nv*2]
 * (either may be NULL) are indexed by the scene's triangle indices (object
 * space in a two-level scene).  Interpolation at barycentrics (b1, b2):
 * ((w0 a0 + b1 a1) + b2 a2) with w0 = (1 - b1) - b2.  Shading normal: the
 * interpolated normal, mapped by the columns of w2o's linear part in a
 * two-level scene, normalised and turned to the geometric normal's side
 * (the geometric normal if the interpolant is zero or not finite).  With
 * normals, the BSDF frame is the shading normal turned to the outgoing
 * direction's side; a vertex whose outgoing direction is below its shading
 * horizon scatters nothing, and light and continuation directions on the
 * wrong geometric side for their lobe (reflection: the outgoing side,
 * transmission: the other) are dropped.  Checker texture: with (u, v)
 * interpolated, the albedo is scaled by 1/4 where floor(u f) + floor(v f)
 * is odd (f the material's checker frequency).  Call after pt_load_scene
 * (which clears them) and before pt_build_bvh; NULL desc or both arrays
 * NULL removes them.  PT_EINVAL on a count mismatch or non-finite value. */
typedef struct {
    int32_t nv;
    const float* normals;
    const float* uvs;
} pt_attributes_desc;
pt_status pt_set_attributes(pt_ctx* ctx, const pt_attributes_desc* attributes);

/* BVH build options (NULL = defaults). */
typedef struct {
    int32_t max_leaf;  /* triangles per leaf, 1..8 (0 = default 1: one triangle per leaf
                          keeps the leaf step uniform across a wave) */
    int32_t threads;   /* host threads for the build (0 = hardware concurrency) */
} pt_bvh_opts;

/* Filled by pt_build_bvh: sizes of the device buffers of pt_scene_buffers. */
typedef struct {
    int64_t node_count, node_bytes;  /* BVH4 nodes, 80 B each (half-precision child boxes) */
    int64_t tri_bytes;               /* 48 B per triangle, leaf order, plus 32 B of padding */
    int64_t light_count, light_bytes;/* 16 B per light (leaf-order index, CDF word, input index, 0),
                                        then the input ids of the 64 largest triangles */
    int64_t material_bytes;          /* 16 B per material */
    int64_t instance_count, instance_bytes; /* two-level scenes: 112 B per instance record */
    int64_t attribute_bytes;         /* vertex attributes: 64 B per triangle, leaf order (0 without) */
    int32_t depth;                   /* BVH4 levels */
    int32_t stack_entries;           /* traversal stack entries needed */
    double build_seconds;
} pt_bvh_info;

/* Caller-allocated device buffers, each at least the size pt_build_bvh
 * reported and 256-byte aligned.  nodes/tris/lights/materials are written
 * by pt_bind_scene (upload on the stream).  albedo and emission are
 * float[nt*3] device arrays in input triangle order that the kernels read
 * at every render: they are the differentiable parameters; pt_bind_scene
 * fills them from the loaded scene when upload_params != 0. */
typedef struct {
    void* nodes;
    void* tris;
    void* lights;
    void* materials;
    float* albedo;
    float* emission;
    int32_t upload_params;
    void* instances;  /* instance records (two-level scenes; may be NULL for a flat scene) */
    void* attributes; /* vertex attribute records (may be NULL without attributes) */
} pt_scene_buffers;

/* Pinhole camera: eye, target, up, vertical field of view (degrees),
 * image size.  Row py = 0 is the top of the image. */
typedef struct {
    double eye[3], target[3], up[3];
    double vfov_deg;
    int32_t width, height;
} pt_camera;

/* Per-render arguments.  max_depth = number of scattering vertices
 * (emission found after the last one is still counted); rr_start < 0
 * disables Russian roulette, else it applies from that vertex on.
 * block = threads per workgroup (64..256, multiple of 64; 0 = default 256);
 * grid_mult = persistent workgroups per compute unit (0 = default 8);
 * sort_threshold: with PT_FLAG_SORT_MATERIAL (PT_FLAG_SORT_RAYS), a
 * bounce's shade (extend) queue is sorted only when it holds at least this
 * many paths;
 * stack_lds: traversal stack entries kept in LDS per lane, 8/16/24/32
 * (0 = default 8); deeper entries spill to the workspace; (stack_lds + 1)
 * x 8 bytes per thread of LDS plus 12 KiB of light table must fit one
 * workgroup's LDS (PT_EINVAL otherwise);
 * tail_threshold: wavefront hybrid tail, a bounce whose queue holds fewer
 * than this many paths finishes them in place, megakernel style, inside the
 * shade stage (0 = off; the image is the same bit for bit);
 * tail_bounce: when > 0, the hybrid tail finishes every path still running
 * at bounce tail_bounce (1 .. max_depth) whatever the queue size, and no
 * stage of a later bounce is enqueued (0 = off; same image bit for bit);
 * sampler: camera jitter, PT_SAMPLER_PHILOX (words of the path's counter)
 * or PT_SAMPLER_HALTON (the ray generation sampler of Sec. 2.3: the
 * Halton(2,3) point of the pixel's sample index frame*spp + s, radical
 * inverses truncated to 24 bits, Cranley-Patterson rotated per pixel by
 * 24-bit offsets from the Philox block of the reserved sample index
 * 0xFFFFFFFF, modulo 1); every later dimension of the path stays Philox.
 * Any other value is PT_EINVAL.
 * tail_spread: 1 = the hybrid tail spreads its queue over as many waves as
 * the device holds at once (partly filled waves, more latency hidden: faster
 * when a frame runs alone), 0 = full waves (fewer instructions: faster with
 * frames in flight); same image bit for bit.
 * mega_waves: the megakernel's occupancy, 4 (0 = default) or 5 waves per
 * SIMD (more registers spilled: slower frame by frame, faster with frames in
 * flight); same image bit for bit. */
typedef struct {
    int32_t spp, max_depth;
    uint64_t seed;
    uint32_t frame;
    uint32_t job;
    int32_t nee, rr_start;
    int32_t mode;
    int32_t flags;
    int32_t block, grid_mult;
    uint32_t sort_threshold;
    int32_t stack_lds;
    uint32_t tail_threshold;
    int32_t tail_bounce;
    int32_t sampler;
    int32_t tail_spread;
    int32_t mega_waves;
} pt_render_args;

/* Library version (major * 10000 + minor * 100 + patch). */
int32_t pt_version(void);
/* Message of the last failing call on this thread ("" if none). */
const char* pt_last_error(void);

/* Create a context on HIP device `device`; device < 0 creates a host-only
 * context (scene load and BVH build only; rendering returns PT_ESTATE).
 * PT_EHIP if the device does not exist or HIP is unavailable. */
pt_status pt_create(pt_ctx** out, int32_t device);
pt_status pt_destroy(pt_ctx* ctx);

/* Copy and validate the scene (replaces any previous one). */
pt_status pt_load_scene(pt_ctx* ctx, const pt_scene_desc* scene);

/* CPU build of the acceleration structure (paper Sec. 3 builds BLAS/TLAS
 * through the driver; here a binned-SAH binary BVH collapsed to a 4-wide
 * BVH with 80-byte nodes), the leaf-order triangle array and the
 * area-proportional light CDF.  Synchronous, host only. */
pt_status pt_build_bvh(pt_ctx* ctx, const pt_bvh_opts* opts, pt_bvh_info* info);

/* Host copies of the built buffers (each may be NULL), sizes as reported
 * (the triangle array without its 32 B of padding: 48 B per triangle). */
pt_status pt_get_bvh(pt_ctx* ctx, void* nodes, void* tris, void* lights, void* materials);

/* Upload the built buffers into the caller's device buffers on `stream`
 * and remember the pointers for later renders.  The buffers must stay
 * allocated while the context renders with them. */
pt_status pt_bind_scene(pt_ctx* ctx, const pt_scene_buffers* buffers, void* stream);

pt_status pt_set_camera(pt_ctx* ctx, const pt_camera* camera);

/* Device workspace (bytes) a render with these arguments needs, for the
 * camera currently set: wavefront path state, queues and counters, and
 * the traversal stack overflow area (two of them in PT_MODE_WAVE: the
 * shadow stage has its own). */
pt_status pt_workspace_size(pt_ctx* ctx, const pt_render_args* args, uint64_t* bytes);

/* Render one frame (paper Sec. 2.2 megakernel / Sec. 2.3 wavefront).
 * image_out: float[H][W][3] device, this frame's per-pixel mean over spp.
 * accum_inout (may be NULL): float[H][W][3] device running average
 * (paper Sec. 2.3 accumulation): frame 0 stores the frame, frame n > 0
 * stores acc + (I - acc) / (n + 1).
 * workspace: device memory of at least pt_workspace_size bytes.
 * In PT_MODE_WAVE each bounce's shadow stage runs on an internal stream
 * of the context (default priority, created on first use), forked from
 * `stream` after the shade stage and joined before the next one; the
 * call's results are complete when `stream` reaches its end, and the
 * image is the same bit for bit as with every stage on `stream`. */
pt_status pt_render_frame(pt_ctx* ctx, const pt_render_args* args, float* image_out,
                          float* accum_inout, void* workspace, uint64_t workspace_bytes,
                          void* stream);

/* For callers that cannot allocate device memory or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): pt_render_frame with the megakernel (args->mode must be
 * PT_MODE_MEGA, else PT_EUNSUPPORTED; PT_FLAG_PROFILE is PT_EINVAL), whose
 * counters, pixel cursor and traversal stack overflow area live in a scratch
 * array of 64 MiB that the library holds on each GPU it runs on (looked up
 * by pt_create) until the process ends.  The caller passes the image and the
 * optional running average as in pt_render_frame; the call allocates
 * nothing.  PT_ENOMEM if the frame's launch configuration needs more scratch
 * than that (the traversal stack overflow area grows with grid_mult x block
 * x (BVH stack entries - stack_lds) x 8 bytes).  Every call on a GPU shares
 * that GPU's array and leaves its contents behind (pt_frame_stats_get reads
 * the last call's counters): calls that overlap on one GPU, from any
 * context, race.  The image equals pt_render_frame's bit for bit. */
pt_status pt_render_frame_noalloc(pt_ctx* ctx, const pt_render_args* args, float* image_out, float* accum_inout,
                                  void* stream);

/* Progressive rendering with F frames in flight: frames args->frame,
 * ..., args->frame + n_frames - 1, each exactly as pt_render_frame renders
 * it.  A frame's stages run on one of F internal streams of the context
 * (default priority, created on first use) while the frames before it
 * finish on the others, so that the short last bounces of one frame overlap
 * the first bounces of the next; the per-frame accumulation runs on
 * `stream` in frame order.  F is fixed when the context is created: two
 * less than the hardware queues HIP gives the process (the environment
 * variable GPU_MAX_HW_QUEUES, 4 when unset; it must be set before the
 * process first uses HIP to take effect), between 3 and 8.  Work enqueued on `stream` before the call precedes every
 * frame; the call's results are complete when `stream` reaches its end.
 * image_out receives each frame's image in turn (the last one remains);
 * accum_inout (may be NULL) is updated as by n_frames calls of
 * pt_render_frame, bit for bit.  workspace: pt_frames_workspace_size bytes
 * (F frame slots), 256-byte aligned.  PT_EINVAL with PT_FLAG_PROFILE.
 * Calls that overlap on one context race. */
pt_status pt_frames_workspace_size(pt_ctx* ctx, const pt_render_args* args, uint64_t* bytes);
pt_status pt_render_frames(pt_ctx* ctx, const pt_render_args* args, int32_t n_frames, float* image_out,
                           float* accum_inout, void* workspace, uint64_t workspace_bytes, void* stream);

/* Path-replay adjoint of one frame: ACCUMULATES (+=) into d_albedo and
 * d_emission (float[nt*3] device, input triangle order) the gradient of
 * sum_p sum_c d_image[p][c] * I[p][c] for the fixed-sample estimator defined
 * by (seed, frame, spp, job).  Each path is replayed twice from its random
 * numbers: a first pass over all paths keeps only each path's radiance (16
 * bytes per path in the workspace), a second pass replays them again and
 * adds the gradients; by default no vertex is stored.  args->mode selects how the
 * first pass runs: PT_MODE_MEGA as one megakernel-style kernel, PT_MODE_WAVE
 * as the wavefront stages with the frame's wavefront options (hybrid tail,
 * sorts), whose per-path radiance is the same bit for bit; the second pass
 * is one kernel either way.  With PT_FLAG_KEEP_HITS the first pass also
 * keeps every vertex's intersection and light-sample visibility and the
 * second traces no ray (same gradients, 9 bytes per path vertex of
 * workspace).
 * workspace: at least pt_backward_workspace_size bytes (path cursors, the
 * per-path radiance, the wavefront buffers in PT_MODE_WAVE, the kept
 * records with PT_FLAG_KEEP_HITS, the traversal stack overflow area),
 * 256-byte aligned.
 * PT_EINVAL if Russian roulette is on (its survival probability depends on
 * the albedo). */
pt_status pt_backward_workspace_size(pt_ctx* ctx, const pt_render_args* args, uint64_t* bytes);
pt_status pt_render_backward(pt_ctx* ctx, const pt_render_args* args, const float* d_image,
                             float* d_albedo, float* d_emission, void* workspace,
                             uint64_t workspace_bytes, void* stream);

/* Statistics of the last frame rendered (synchronises the stream).
 * Stages (index k): 0 raygen, 1 extend, 2 shade, 3 shadow, 4 accumulate,
 * 5 megakernel, 6 sort, 7 adjoint replay B (gradients), 8 hybrid tail,
 * 9 adjoint replay A (path radiance), 10 promote (the two-slot count
 * buffer of PT_FLAG_TWO_SLOT).
 *   stage_ms[k], launches[k]: HIP-event time and launch count per stage,
 *     filled only when the frame ran with PT_FLAG_PROFILE (else 0).
 *   stage_items[k]: work items the stage's launches processed (paths for
 *     raygen, accumulate pixels, queued rays for extend / shade / shadow /
 *     tail, paths for the megakernel and the adjoint); always filled.
 *   stage_bytes[k]: the stage's algorithmic path-state bytes (reads +
 *     writes of queue records, radiance and image buffers a stage must move;
 *     scene data excluded; conditional radiance updates of shade and shadow
 *     excluded, so a lower bound there); always filled.
 *   node_visits[k], tri_tests[k]: BVH node visits (four child boxes tested
 *     each) and ray/triangle tests of the traversal stages (extend, shadow,
 *     hybrid tail, megakernel), filled when the frame ran with
 *     PT_FLAG_COUNT_WORK (else 0).
 *   extension_rays, shadow_rays: rays traced by the frame (wavefront stages
 *   and hybrid tail, or megakernel; for the adjoint the rays of the paths,
 *   which replay A and replay B each trace once).
 * PT_EOVERFLOW if a traversal stack overflowed during the frame. */
#define PT_NSTAGES 11
typedef struct {
    double stage_ms[PT_NSTAGES];
    int64_t launches[PT_NSTAGES];
    int64_t stage_items[PT_NSTAGES];
    double stage_bytes[PT_NSTAGES];
    int64_t node_visits[PT_NSTAGES], tri_tests[PT_NSTAGES];
    int64_t extension_rays, shadow_rays;
} pt_frame_stats;
pt_status pt_frame_stats_get(pt_ctx* ctx, pt_frame_stats* stats);

/* Batched rendering (many views and scenes of uneven size in one
 * persistent wavefront).  Each job names a context (scene bound, camera
 * set; all on one device), its render arguments (spp, max_depth, seed,
 * frame, nee, rr_start; args.job keys its random numbers, so a job renders
 * exactly what pt_render_frame renders with the same arguments) and its
 * device image float[H][W][3].  All jobs' paths share one pool of
 * pool_capacity slots refilled every iteration (path regeneration). */
typedef struct {
    pt_ctx* ctx;
    pt_render_args args;
    float* image_out;
} pt_job;

typedef struct {
    uint32_t pool_capacity;  /* path slots (0 = 2^21) */
    int32_t block, grid_mult;/* as in pt_render_args (0 = defaults) */
    int32_t stack_lds;       /* as in pt_render_args (0 = default) */
    int32_t iters_per_graph; /* iterations captured per graph launch, even (0 = 8) */
    int32_t use_graph;       /* 1 = capture and replay a hipGraph, 0 = plain launches */
    int32_t pools;           /* pools run concurrently, 1..4 (0 = 1): the jobs are split into
                                pools of about equal path counts, each with pool_capacity / pools
                                slots, its own stream and graph; no pool may be left without a job */
} pt_batch_opts;

typedef struct {
    double seconds;          /* host wall time of the whole batch */
    int64_t path_samples;    /* sum over jobs of W * H * spp */
    int64_t iterations;      /* pool iterations that did work */
    int64_t launches;        /* graph launches (or iterations without a graph) */
} pt_batch_result;

/* Device workspace of a batch (bytes): job table, control block, pool
 * state, per-path radiance of every job, traversal stack overflow. */
pt_status pt_batch_workspace_size(const pt_job* jobs, int32_t n_jobs, const pt_batch_opts* opts,
                                  uint64_t* bytes);

/* Render all jobs; returns when every image is written (synchronous).
 * job_ms (may be NULL): per job, device time from the start of the batch
 * to the moment its last path finished, in milliseconds. */
pt_status pt_render_batch(const pt_job* jobs, int32_t n_jobs, const pt_batch_opts* opts, void* workspace,
                          uint64_t workspace_bytes, void* stream, double* job_ms, pt_batch_result* result);

/* Wait for all work the context enqueued on `stream`. */
pt_status pt_sync(pt_ctx* ctx, void* stream);

#ifdef __cplusplus
}
#endif
#endif
